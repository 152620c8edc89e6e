"""Python binding of the gfx950 p-dit library (``include/pdit.h``).

Argument marshalling only: every step of the sweep runs in the library's HIP
kernels.  Tensors are torch CUDA (ROCm) tensors on the context's device;
PyTorch provides device memory and the stream, nothing else.  If the built
library is missing, loading fails loudly; there is no CPU fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import os
import weakref

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpdit.so")

PDIT_OK = 0
STATUS = {0: "PDIT_OK", -1: "PDIT_EINVAL", -2: "PDIT_ENOTSYM", -3: "PDIT_EBADPERM",
          -4: "PDIT_EOVERFLOW", -5: "PDIT_ENOMEM", -6: "PDIT_EDEVICE", -7: "PDIT_EBETA",
          -8: "PDIT_ESTATE", -9: "PDIT_ECHECK"}
NMAX = 512

RECOMPUTE = {"auto": 0, "plain": 1, "i8": 2, "bf16": 3, "split": 4}
SWEEP = {"auto": 0, "plain": 1, "fast": 2, "clique": 3, "large": 4, "reg": 5}
PT_SCHEDULE = {"auto": 0, "periodic": 1, "fused": 2}
PT_DYNAMICS = {"sequential": 0, "cupim": 1}


class PditError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code
        self.status = STATUS.get(code, str(code))


class _Opts(C.Structure):
    _fields_ = [("device", C.c_int), ("stream", C.c_void_p), ("recompute", C.c_int),
                ("sweep", C.c_int), ("blocks_per_cu", C.c_int), ("seq_threshold", C.c_int),
                ("paranoid", C.c_int)]


class _Tuning(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int), ("seq_threshold", C.c_int), ("best_ms", C.c_double),
                ("cached", C.c_int)]


class _Counters(C.Structure):
    _fields_ = [("updates", C.c_int64), ("accepted", C.c_int64), ("ties", C.c_int64)]


class _Instance(C.Structure):
    _fields_ = [("N", C.c_int32), ("R", C.c_int32), ("D", C.c_void_p), ("F", C.c_void_p),
                ("perm", C.c_void_p), ("beta", C.c_void_p), ("choices", C.c_void_p),
                ("E_trace", C.c_void_p)]


class _PT(C.Structure):
    _fields_ = [("L", C.c_int32), ("beta", C.c_void_p), ("slot", C.c_void_p),
                ("since_top", C.c_void_p), ("period_sweeps", C.c_int64), ("timeout", C.c_int32),
                ("schedule", C.c_int32), ("dynamics", C.c_int32)]


_lib = None

EXPORTS = ["pdit_default_opts", "pdit_create", "pdit_destroy", "pdit_run_sweeps",
           "pdit_run_sweeps_batch", "pdit_energy", "pdit_best", "pdit_counters",
           "pdit_replica_counters", "pdit_set_sweep_offset", "pdit_get_sweep_offset",
           "pdit_reset", "pdit_sync", "pdit_last_error", "pdit_set_recording",
           "pdit_h_recompute", "pdit_debug_delta", "pdit_debug_choice", "pdit_debug_uniform24",
           "pdit_last_timing", "pdit_autotune", "pdit_last_plan", "pdit_run_pt",
           "pdit_beta_select", "pdit_run_cupim", "pdit_run_sweeps_noalloc", "pdit_debug_H",
           "pdit_debug_delta_replica"]


def load_library(path: str = LIB_PATH):
    """Load ``libpdit.so`` and declare its signatures.  Raises if it is not
    built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_2605_24408_amd.build` "
                           "(the p-dit path has no CPU fallback)")
    L = C.CDLL(path)
    vp, i32, i64, u64 = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64
    L.pdit_default_opts.restype = None
    L.pdit_default_opts.argtypes = [C.POINTER(_Opts)]
    L.pdit_create.argtypes = [C.POINTER(vp), C.POINTER(_Opts)]
    L.pdit_destroy.argtypes = [vp]
    L.pdit_run_sweeps.argtypes = [vp, i32, vp, vp, i32, vp, vp, i64, u64]
    L.pdit_run_sweeps_batch.argtypes = [vp, i32, C.POINTER(_Instance), i64, u64]
    L.pdit_run_pt.argtypes = [vp, i32, vp, vp, i32, vp, C.POINTER(_PT), i64, u64]
    L.pdit_run_cupim.argtypes = [vp, i32, vp, vp, i32, vp, vp, i64, u64]
    L.pdit_beta_select.argtypes = [vp, i32, vp, vp, i32, vp, vp, i32, i64, u64, i32, i32, vp, vp,
                                   vp]
    L.pdit_energy.argtypes = [vp, vp]
    L.pdit_best.argtypes = [vp, vp, vp]
    L.pdit_counters.argtypes = [vp, C.POINTER(_Counters)]
    L.pdit_replica_counters.argtypes = [vp, vp]
    L.pdit_set_sweep_offset.argtypes = [vp, u64]
    L.pdit_get_sweep_offset.argtypes = [vp, C.POINTER(u64)]
    L.pdit_reset.argtypes = [vp]
    L.pdit_sync.argtypes = [vp]
    L.pdit_last_error.restype = C.c_char_p
    L.pdit_last_error.argtypes = [vp]
    L.pdit_set_recording.argtypes = [vp, vp, vp]
    L.pdit_h_recompute.argtypes = [vp, i32, vp, vp, i32, vp, C.c_int, vp, vp]
    L.pdit_debug_delta.argtypes = [vp, i32, vp, vp, i32, vp, i32, vp]
    L.pdit_debug_choice.argtypes = [vp, i32, i32, vp, vp, vp, vp, vp]
    L.pdit_debug_uniform24.argtypes = [vp, i32, vp, u64, vp]
    L.pdit_last_timing.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.pdit_autotune.argtypes = [vp, i32, C.POINTER(_Instance), i64, u64, C.POINTER(_Tuning)]
    L.pdit_last_plan.argtypes = [vp, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.pdit_debug_H.argtypes = [vp, i32, i32, vp]
    L.pdit_debug_delta_replica.argtypes = [vp, i32, i32, i32, vp]
    L.pdit_run_sweeps_noalloc.argtypes = [C.POINTER(_Opts), i32, vp, vp, i32, vp, vp, i64, u64,
                                          u64, C.c_int, vp, vp, vp, vp, C.c_char_p, i32]
    for name in EXPORTS:
        f = getattr(L, name)
        if name not in ("pdit_default_opts", "pdit_last_error"):
            f.restype = C.c_int
    _lib = L
    return L


def _ptr(t: torch.Tensor | None):
    return None if t is None else C.c_void_p(t.data_ptr())


def _check_dev(t: torch.Tensor, dtype, name: str, device: torch.device):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must live on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def run_sweeps_noalloc(D: torch.Tensor, F: torch.Tensor, perm: torch.Tensor, beta: torch.Tensor,
                       seed: int, sweep_offset: int, E: torch.Tensor, E_best: torch.Tensor,
                       perm_best: torch.Tensor, counters: torch.Tensor, init_best: bool = True,
                       stream: torch.cuda.Stream | None = None, sweep: str = "auto",
                       recompute: str = "auto", seq_threshold: int = -1) -> None:
    """pdit_run_sweeps_noalloc: the sweeps of ``Pdit.run_sweeps`` with the
    library's static device scratch instead of a context's buffers; the
    caller's E [R], E_best [R], perm_best [R, N] and counters [R, 3]
    receive the results (E_best and perm_best in/out unless init_best)."""
    L = load_library()
    device = perm.device
    N = int(D.shape[0])
    R = int(perm.shape[0])
    for t, dt, nm in ((D, torch.int32, "D"), (F, torch.int32, "F"), (perm, torch.int32, "perm"),
                      (beta, torch.float32, "beta"), (E, torch.int64, "E"),
                      (E_best, torch.int64, "E_best"), (perm_best, torch.int32, "perm_best"),
                      (counters, torch.int64, "counters")):
        _check_dev(t, dt, nm, device)
    if tuple(D.shape) != (N, N) or tuple(F.shape) != (N, N) or tuple(perm.shape) != (R, N):
        raise ValueError("D and F must be N x N and perm R x N")
    if (tuple(E.shape) != (R,) or tuple(E_best.shape) != (R,) or tuple(perm_best.shape) != (R, N)
            or tuple(counters.shape) != (R, 3)):
        raise ValueError("outputs must be E [R], E_best [R], perm_best [R, N], counters [R, 3]")
    if stream is None:
        stream = torch.cuda.current_stream(device)
    o = _Opts()
    L.pdit_default_opts(C.byref(o))
    o.device = device.index or 0
    o.stream = stream.cuda_stream
    o.recompute = RECOMPUTE[recompute]
    o.sweep = SWEEP[sweep]
    o.seq_threshold = seq_threshold
    err = C.create_string_buffer(256)
    rc = L.pdit_run_sweeps_noalloc(C.byref(o), N, _ptr(D), _ptr(F), R, _ptr(perm), _ptr(beta),
                                   int(beta.numel()), int(seed), int(sweep_offset),
                                   int(bool(init_best)), _ptr(E), _ptr(E_best), _ptr(perm_best),
                                   _ptr(counters), err, 256)
    if rc != PDIT_OK:
        raise PditError(rc, err.value.decode())


# Contexts still open at interpreter exit are closed by an exit hook, while
# the HIP runtime and torch are intact: a context left to garbage collection
# during interpreter finalization would call pdit_destroy (hipSetDevice,
# hipStreamSynchronize, hipFree, ...) in whatever order the runtime's own
# teardown has reached by then.
_open_contexts: "weakref.WeakSet[Pdit]" = weakref.WeakSet()


@atexit.register
def _close_open_contexts():
    for ctx in list(_open_contexts):
        try:
            ctx.close()
        except Exception:
            pass


class Pdit:
    """A library context (``pdit_create``) bound to one device and stream.
    ``paranoid``: every sweep of ``run_sweeps`` is its own launch and is
    rechecked against Eq. 1 recomputed from the permutations (PditError
    PDIT_ECHECK on a mismatch; no recording in this mode)."""

    def __init__(self, device: int = 0, stream: torch.cuda.Stream | None = None,
                 recompute: str = "auto", sweep: str = "auto", blocks_per_cu: int = 0,
                 seq_threshold: int = -1, paranoid: bool = False):
        self._L = load_library()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        o = _Opts()
        self._L.pdit_default_opts(C.byref(o))
        o.device = device
        o.stream = stream.cuda_stream
        o.recompute = RECOMPUTE[recompute]
        o.sweep = SWEEP[sweep]
        o.blocks_per_cu = blocks_per_cu
        o.seq_threshold = seq_threshold
        o.paranoid = int(bool(paranoid))
        h = C.c_void_p()
        rc = self._L.pdit_create(C.byref(h), C.byref(o))
        if rc != PDIT_OK:
            raise PditError(rc, "pdit_create failed")
        self._h = h
        self._last = None   # (R_total, perm_total, N) of the last run
        _open_contexts.add(self)

    # -- lifetime ---------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            self._L.pdit_destroy(self._h)
            self._h = None
        _open_contexts.discard(self)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _rc(self, rc: int):
        if rc != PDIT_OK:
            msg = self._L.pdit_last_error(self._h)
            raise PditError(rc, msg.decode() if msg else "")

    # -- runs -------------------------------------------------------------
    def run_sweeps(self, D: torch.Tensor, F: torch.Tensor, perm: torch.Tensor,
                   beta: torch.Tensor, seed: int) -> None:
        """pdit_run_sweeps: len(beta) sweeps on every row of perm (in/out)."""
        N = int(D.shape[0])
        for t, dt, nm in ((D, torch.int32, "D"), (F, torch.int32, "F"),
                          (perm, torch.int32, "perm"), (beta, torch.float32, "beta")):
            _check_dev(t, dt, nm, self.device)
        if tuple(D.shape) != (N, N) or tuple(F.shape) != (N, N):
            raise ValueError("D and F must be N x N")
        if perm.dim() != 2 or perm.shape[1] != N:
            raise ValueError("perm must be R x N")
        R = int(perm.shape[0])
        self._rc(self._L.pdit_run_sweeps(self._h, N, _ptr(D), _ptr(F), R, _ptr(perm),
                                         _ptr(beta), int(beta.numel()), int(seed)))
        self._last = (R, R * N, N)

    def _instances(self, instances, n_sweeps: int | None):
        """instances: sequence of (D, F, perm, beta) tensors, optionally
        followed by recording buffers (choices int32 [R, T, N] or None,
        E_trace int64 [R, T] or None); every beta has the same length."""
        arr = (_Instance * len(instances))()
        T = None
        for k, item in enumerate(instances):
            D, F, perm, beta = item[:4]
            ch = item[4] if len(item) > 4 else None
            tr = item[5] if len(item) > 5 else None
            for t, dt, nm in ((D, torch.int32, "D"), (F, torch.int32, "F"),
                              (perm, torch.int32, "perm"), (beta, torch.float32, "beta")):
                _check_dev(t, dt, nm, self.device)
            N = int(D.shape[0])
            if tuple(D.shape) != (N, N) or tuple(F.shape) != (N, N) or perm.dim() != 2 \
                    or perm.shape[1] != N:
                raise ValueError(f"instance {k}: D, F must be N x N and perm R x N")
            if T is None:
                T = int(beta.numel())
            elif int(beta.numel()) != T:
                raise ValueError("every instance needs a beta schedule of the same length")
            R = int(perm.shape[0])
            if ch is not None:
                _check_dev(ch, torch.int32, "choices", self.device)
                if tuple(ch.shape) != (R, T, N):
                    raise ValueError(f"instance {k}: choices must be R x T x N")
            if tr is not None:
                _check_dev(tr, torch.int64, "E_trace", self.device)
                if tuple(tr.shape) != (R, T):
                    raise ValueError(f"instance {k}: E_trace must be R x T")
            arr[k] = _Instance(N, R, D.data_ptr(), F.data_ptr(), perm.data_ptr(),
                               beta.data_ptr(), None if ch is None else ch.data_ptr(),
                               None if tr is None else tr.data_ptr())
        return arr, (T if n_sweeps is None else n_sweeps)

    def run_pt(self, D: torch.Tensor, F: torch.Tensor, perm: torch.Tensor, beta: torch.Tensor,
               slot: torch.Tensor, since_top: torch.Tensor, n_periods: int, period_sweeps: int,
               timeout: int, seed: int, schedule: str = "auto",
               dynamics: str = "sequential") -> None:
        """pdit_run_pt: parallel tempering over sets of L = len(beta) rows of
        perm (slot, since_top and perm in/out); schedule "auto", "periodic"
        (a launch per period) or "fused" (every period in one launch);
        dynamics "sequential" (sweeps) or "cupim" (concurrent updates)."""
        N = int(D.shape[0])
        for t, dt, nm in ((D, torch.int32, "D"), (F, torch.int32, "F"), (perm, torch.int32, "perm"),
                          (beta, torch.float32, "beta"), (slot, torch.int32, "slot"),
                          (since_top, torch.int32, "since_top")):
            _check_dev(t, dt, nm, self.device)
        R = int(perm.shape[0])
        pt = _PT(int(beta.shape[0]), _ptr(beta), _ptr(slot), _ptr(since_top), int(period_sweeps),
                 int(timeout), PT_SCHEDULE[schedule], PT_DYNAMICS[dynamics])
        self._rc(self._L.pdit_run_pt(self._h, N, _ptr(D), _ptr(F), R, _ptr(perm), C.byref(pt),
                                     int(n_periods), int(seed)))
        self._last = (R, R * N, N)

    def run_cupim(self, D: torch.Tensor, F: torch.Tensor, perm: torch.Tensor,
                  beta: torch.Tensor, seed: int) -> None:
        """pdit_run_cupim: len(beta) concurrent-update iterations on every
        row of perm (in/out)."""
        N = int(D.shape[0])
        for t, dt, nm in ((D, torch.int32, "D"), (F, torch.int32, "F"),
                          (perm, torch.int32, "perm"), (beta, torch.float32, "beta")):
            _check_dev(t, dt, nm, self.device)
        if perm.dim() != 2 or perm.shape[1] != N:
            raise ValueError("perm must be R x N")
        R = int(perm.shape[0])
        self._rc(self._L.pdit_run_cupim(self._h, N, _ptr(D), _ptr(F), R, _ptr(perm), _ptr(beta),
                                        int(beta.numel()), int(seed)))
        self._last = (R, R * N, N)

    def beta_select(self, D: torch.Tensor, F: torch.Tensor, perm: torch.Tensor,
                    grid: torch.Tensor, trial_sweeps: int, seed: int, L: int,
                    level_pct: int = 40):
        """pdit_beta_select: fixed-beta trials on the grid from the rows of
        perm (unchanged), the low end's level level_pct percent of the
        range above the minimum; returns (E_sum [G] int64, ladder [L]
        float32, range [2] int32 = (lo, hi))."""
        N = int(D.shape[0])
        for t, dt, nm in ((D, torch.int32, "D"), (F, torch.int32, "F"), (perm, torch.int32, "perm"),
                          (grid, torch.float32, "grid")):
            _check_dev(t, dt, nm, self.device)
        R, G = int(perm.shape[0]), int(grid.numel())
        E_sum = torch.empty(G, dtype=torch.int64, device=self.device)
        ladder = torch.empty(max(int(L), 1), dtype=torch.float32, device=self.device)
        rng = torch.empty(2, dtype=torch.int32, device=self.device)
        self._rc(self._L.pdit_beta_select(self._h, N, _ptr(D), _ptr(F), R, _ptr(perm), _ptr(grid),
                                          G, int(trial_sweeps), int(seed), int(L),
                                          int(level_pct), _ptr(E_sum), _ptr(ladder), _ptr(rng)))
        self._last = (R * G, R * G * N, N)
        return E_sum, ladder, rng

    def run_sweeps_batch(self, instances, seed: int) -> None:
        """pdit_run_sweeps_batch over (D, F, perm, beta[, choices, E_trace])
        tensors of uneven N."""
        arr, T = self._instances(instances, None)
        self._rc(self._L.pdit_run_sweeps_batch(self._h, len(instances), arr, int(T), int(seed)))
        R = sum(int(x[2].shape[0]) for x in instances)
        PT = sum(int(x[2].numel()) for x in instances)
        self._last = (R, PT, 0)

    def autotune(self, instances, n_trial_sweeps: int, seed: int) -> dict:
        """pdit_autotune: picks blocks per CU and the sequential threshold
        (looked up in, or appended to, the file PDIT_AUTOTUNE_CACHE names)."""
        arr, _ = self._instances(instances, None)
        t = _Tuning()
        self._rc(self._L.pdit_autotune(self._h, len(instances), arr, int(n_trial_sweeps),
                                       int(seed), C.byref(t)))
        return {"blocks_per_cu": t.blocks_per_cu, "seq_threshold": t.seq_threshold,
                "best_ms": t.best_ms, "cached": bool(t.cached)}

    def energy(self) -> torch.Tensor:
        out = torch.empty(self._last[0], dtype=torch.int64, device=self.device)
        self._rc(self._L.pdit_energy(self._h, _ptr(out)))
        return out

    def best(self) -> tuple[torch.Tensor, torch.Tensor]:
        R, PT, N = self._last
        E = torch.empty(R, dtype=torch.int64, device=self.device)
        P = torch.empty(PT, dtype=torch.int32, device=self.device)
        self._rc(self._L.pdit_best(self._h, _ptr(E), _ptr(P)))
        return E, (P.view(R, N) if N else P)

    def counters(self) -> dict:
        c = _Counters()
        self._rc(self._L.pdit_counters(self._h, C.byref(c)))
        return {"updates": c.updates, "accepted": c.accepted, "ties": c.ties}

    def replica_counters(self) -> torch.Tensor:
        out = torch.empty((self._last[0], 3), dtype=torch.int64, device=self.device)
        self._rc(self._L.pdit_replica_counters(self._h, _ptr(out)))
        return out

    def last_timing(self) -> tuple[float, float]:
        """(recompute_ms, sweep_ms) of the last run, from HIP events on the
        context's stream."""
        a, b = C.c_double(), C.c_double()
        self._rc(self._L.pdit_last_timing(self._h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def last_plan(self) -> dict:
        """Kernel, on-chip size class and recompute mode of the last run."""
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        self._rc(self._L.pdit_last_plan(self._h, C.byref(a), C.byref(b), C.byref(c)))
        inv = {v: k for k, v in RECOMPUTE.items()}
        return {"sweep": {1: "plain", 2: "fast", 3: "clique", 4: "large", 5: "reg"}[a.value],
                "size_class": b.value,
                "recompute": inv[c.value]}

    def set_sweep_offset(self, offset: int):
        self._rc(self._L.pdit_set_sweep_offset(self._h, int(offset)))

    def get_sweep_offset(self) -> int:
        v = C.c_uint64()
        self._rc(self._L.pdit_get_sweep_offset(self._h, C.byref(v)))
        return int(v.value)

    def reset(self):
        self._rc(self._L.pdit_reset(self._h))

    def sync(self):
        self._rc(self._L.pdit_sync(self._h))

    def set_recording(self, choices: torch.Tensor | None = None,
                      E_trace: torch.Tensor | None = None):
        self._rc(self._L.pdit_set_recording(self._h, _ptr(choices), _ptr(E_trace)))

    # -- single steps -----------------------------------------------------
    def h_recompute(self, D, F, perm, mode: str = "plain", with_H: bool = True):
        N = int(D.shape[0])
        R = int(perm.shape[0])
        for t, dt, nm in ((D, torch.int32, "D"), (F, torch.int32, "F"), (perm, torch.int32, "perm")):
            _check_dev(t, dt, nm, self.device)
        H = torch.empty((R, N, N), dtype=torch.int64, device=self.device) if with_H else None
        E = torch.empty(R, dtype=torch.int64, device=self.device)
        self._rc(self._L.pdit_h_recompute(self._h, N, _ptr(D), _ptr(F), R, _ptr(perm),
                                          RECOMPUTE[mode], _ptr(H), _ptr(E)))
        return H, E

    def debug_delta(self, D, F, perm, r: int) -> torch.Tensor:
        N = int(D.shape[0])
        R = int(perm.shape[0])
        out = torch.empty((R, N), dtype=torch.int64, device=self.device)
        self._rc(self._L.pdit_debug_delta(self._h, N, _ptr(D), _ptr(F), R, _ptr(perm), int(r),
                                          _ptr(out)))
        return out

    def debug_H(self, inst: int, replica: int, N: int) -> torch.Tensor:
        """pdit_debug_H: H = D F[p,p] (int64 N x N) of a replica of the last run."""
        H = torch.empty((N, N), dtype=torch.int64, device=self.device)
        self._rc(self._L.pdit_debug_H(self._h, int(inst), int(replica), _ptr(H)))
        return H

    def debug_delta_replica(self, inst: int, replica: int, r: int, N: int) -> torch.Tensor:
        """pdit_debug_delta_replica: Eq. 3 for location r of a replica of the last run."""
        out = torch.empty(N, dtype=torch.int64, device=self.device)
        self._rc(self._L.pdit_debug_delta_replica(self._h, int(inst), int(replica), int(r),
                                                  _ptr(out)))
        return out

    def debug_choice(self, delta: torch.Tensor, beta: torch.Tensor, u24: torch.Tensor):
        M, N = int(delta.shape[0]), int(delta.shape[1])
        _check_dev(delta, torch.int64, "delta", self.device)
        _check_dev(beta, torch.float32, "beta", self.device)
        _check_dev(u24, torch.int32, "u24", self.device)
        choice = torch.full((M,), -1, dtype=torch.int32, device=self.device)
        tie = torch.zeros(M, dtype=torch.int32, device=self.device)
        self._rc(self._L.pdit_debug_choice(self._h, N, M, _ptr(delta), _ptr(beta), _ptr(u24),
                                           _ptr(choice), _ptr(tie)))
        return choice, tie

    def debug_uniform24(self, ctr: torch.Tensor, seed: int) -> torch.Tensor:
        _check_dev(ctr, torch.int32, "ctr", self.device)
        M = int(ctr.shape[0])
        out = torch.empty(M, dtype=torch.int32, device=self.device)
        self._rc(self._L.pdit_debug_uniform24(self._h, M, _ptr(ctr), int(seed), _ptr(out)))
        return out
