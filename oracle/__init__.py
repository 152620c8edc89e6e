"""ctypes front end of the plain CPU oracle (``pdit_oracle.c``).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
benchmark's CPU-baseline leg may use this package; the GPU library never
does.  The oracle shares no code with the GPU path.

``build()`` compiles the C file with gcc (plain -O2, no vector intrinsics,
floating-point contraction off so the double-precision evaluation of Eq. 5
rounds exactly as written).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pdit_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

PO_OK, PO_EINVAL, PO_EMISMATCH, PO_EBADPERM, PO_ENOMEM = 0, -1, -2, -3, -4


def build(force: bool = True) -> str:
    """Compile liboracle.so next to the source."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                        "-fno-fast-math", "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"],
                       check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = C.CDLL(_LIB)
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        u32p = np.ctypeslib.ndpointer(np.uint32, flags="C_CONTIGUOUS")
        f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
        L.po_energy.restype = C.c_int64
        L.po_energy.argtypes = [C.c_int, i32p, i32p, i32p]
        L.po_influence.restype = None
        L.po_influence.argtypes = [C.c_int, i32p, i32p, i32p, i64p]
        for fn in (L.po_delta_eq3, L.po_delta_eq4):
            fn.restype = C.c_int64
            fn.argtypes = [C.c_int, i32p, i32p, i32p, i64p, C.c_int, C.c_int]
        L.po_delta_row.restype = C.c_int
        L.po_delta_row.argtypes = [C.c_int, i32p, i32p, i32p, C.c_int, i64p]
        L.po_philox4x32_10.restype = None
        L.po_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.po_uniform24.restype = C.c_uint32
        L.po_uniform24.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32]
        L.po_gibbs_choice.restype = C.c_int
        L.po_gibbs_choice.argtypes = [C.c_int, i64p, C.c_float, C.c_uint32, C.POINTER(C.c_int),
                                      C.POINTER(C.c_double)]
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        L.po_gibbs_rows.restype = C.c_int
        L.po_gibbs_rows.argtypes = [C.c_int64, C.c_int, i64p, f32p, u32p, i32p, i32p, f64p]
        L.po_sample_choices.restype = C.c_int
        L.po_sample_choices.argtypes = [C.c_int, i64p, C.c_float, C.c_uint64, C.c_uint32,
                                        C.c_uint32, C.c_uint32, C.c_uint32, C.c_int64, i64p]
        L.po_run.restype = C.c_int
        L.po_run.argtypes = [C.c_int, i32p, i32p, C.c_int, C.c_void_p, C.c_int32, i32p, f32p,
                             C.c_int64, C.c_uint64, C.c_uint64, i64p, i64p, i32p, C.c_int, i64p,
                             C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                             C.c_void_p, C.c_void_p, C.c_void_p]
        L.po_brute_min.restype = C.c_int64
        L.po_brute_min.argtypes = [C.c_int, i32p, i32p, C.c_int, i32p]
        L.po_pt_exchange.restype = C.c_int
        L.po_pt_exchange.argtypes = [C.c_int, i64p, i32p, i32p, C.c_int32]
        L.po_run_pt.restype = C.c_int
        L.po_run_pt.argtypes = [C.c_int, i32p, i32p, C.c_int, C.c_int, i32p, f32p, i32p, i32p,
                                C.c_int64, C.c_int64, C.c_int32, C.c_uint64, C.c_uint64,
                                C.c_int32, i64p, i64p, i32p, C.c_int, i64p, C.c_int]
        u8p = np.ctypeslib.ndpointer(np.uint8, flags="C_CONTIGUOUS")
        L.po_cupim_resolve.restype = C.c_int
        L.po_cupim_resolve.argtypes = [C.c_int, i32p, i64p, u8p]
        L.po_run_cupim.restype = C.c_int
        L.po_run_cupim.argtypes = [C.c_int, i32p, i32p, C.c_int, C.c_void_p, C.c_int32, i32p, f32p,
                                   C.c_int64, C.c_uint64, C.c_uint64, i64p, i64p, i32p, C.c_int,
                                   i64p, C.c_void_p, C.c_void_p]
        L.po_beta_rule.restype = C.c_int
        L.po_beta_rule.argtypes = [C.c_int, i64p, f32p, C.c_int, C.c_int, f32p, i32p]
        L.po_beta_select.restype = C.c_int
        L.po_beta_select.argtypes = [C.c_int, i32p, i32p, C.c_int, i32p, f32p, C.c_int, C.c_int64,
                                     C.c_uint64, C.c_int32, C.c_int, C.c_int, i64p, C.c_void_p,
                                     C.c_void_p, C.c_void_p]
        _lib = L
    return _lib


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def energy(D, F, p) -> int:
    """Eq. 1."""
    D, F, p = _i32(D), _i32(F), _i32(p)
    return int(lib().po_energy(D.shape[0], D, F, p))


def influence(D, F, p) -> np.ndarray:
    """Eq. 2 as an [N, N] array indexed (location, facility)."""
    D, F, p = _i32(D), _i32(F), _i32(p)
    N = D.shape[0]
    out = np.zeros((N, N), dtype=np.int64)
    lib().po_influence(N, D, F, p, out)
    return out


def delta_eq3(D, F, p, I, i, j) -> int:
    D, F, p = _i32(D), _i32(F), _i32(p)
    return int(lib().po_delta_eq3(D.shape[0], D, F, p, np.ascontiguousarray(I, np.int64), i, j))


def delta_eq4(D, F, p, I, i, j) -> int:
    D, F, p = _i32(D), _i32(F), _i32(p)
    return int(lib().po_delta_eq4(D.shape[0], D, F, p, np.ascontiguousarray(I, np.int64), i, j))


def delta_row(D, F, p, r) -> np.ndarray:
    D, F, p = _i32(D), _i32(F), _i32(p)
    N = D.shape[0]
    out = np.zeros(N, dtype=np.int64)
    rc = lib().po_delta_row(N, D, F, p, int(r), out)
    if rc != PO_OK:
        raise ValueError(f"po_delta_row failed: {rc}")
    return out


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().po_philox4x32_10(c, k, out)
    return out


def uniform24(seed, r, g, rep, inst) -> int:
    return int(lib().po_uniform24(seed, r, g, rep, inst))


def gibbs_choice(dE, beta, u24) -> tuple[int, bool]:
    """Eq. 5 in double precision: (chosen candidate, tie flag)."""
    k, tie, _ = gibbs_choice_margin(dE, beta, u24)
    return k, tie


def gibbs_choice_margin(dE, beta, u24) -> tuple[int, bool, float]:
    """(chosen candidate, tie flag, distance of tau to the nearest boundary
    between candidates of nonzero weight over Z; inf when there is none)."""
    dE = np.ascontiguousarray(dE, dtype=np.int64)
    tie = C.c_int(0)
    margin = C.c_double(0.0)
    k = lib().po_gibbs_choice(dE.shape[0], dE, np.float32(beta), int(u24), C.byref(tie),
                              C.byref(margin))
    if k < 0:
        raise MemoryError
    return int(k), bool(tie.value), float(margin.value)


def gibbs_rows(dE, beta, u24):
    """Eq. 5 on every row of dE [M, N] with beta[M] and u24[M]: returns
    (choices, tie flags, margins)."""
    dE = np.ascontiguousarray(dE, dtype=np.int64)
    M, N = dE.shape
    beta = np.ascontiguousarray(np.broadcast_to(np.asarray(beta, np.float32), (M,)))
    u24 = np.ascontiguousarray(np.broadcast_to(np.asarray(u24, np.uint32), (M,)))
    sel = np.zeros(M, dtype=np.int32)
    tie = np.zeros(M, dtype=np.int32)
    margin = np.zeros(M, dtype=np.float64)
    rc = lib().po_gibbs_rows(M, N, dE, beta, u24, sel, tie, margin)
    if rc != PO_OK:
        raise RuntimeError(f"po_gibbs_rows failed: {rc}")
    return sel, tie.astype(bool), margin


def sample_choices(dE, beta, seed, r, g0, rep, inst, M) -> np.ndarray:
    dE = np.ascontiguousarray(dE, dtype=np.int64)
    counts = np.zeros(dE.shape[0], dtype=np.int64)
    rc = lib().po_sample_choices(dE.shape[0], dE, np.float32(beta), seed, r, g0, rep, inst,
                                 int(M), counts)
    if rc != PO_OK:
        raise RuntimeError(rc)
    return counts


@dataclass
class RunResult:
    perm: np.ndarray
    E: np.ndarray
    E_best: np.ndarray
    perm_best: np.ndarray
    counters: np.ndarray          # [R, 3]: updates, accepted, ties
    ties: np.ndarray              # [n, 3]: (row, sweep, location)
    choices: np.ndarray | None    # [R, T, N]
    E_trace: np.ndarray | None    # [R, T]
    excused: np.ndarray | None = None  # [R]: forced draws adopted at ties


class OracleMismatch(AssertionError):
    """A forced draw differed from the oracle's own choice off a tie."""

    def __init__(self, row, t, r, own, forced):
        super().__init__(f"draw (row {row}, sweep {t} of the call, location {r}): oracle "
                         f"chose {own}, the other path {forced}, and the oracle saw no tie")
        self.row, self.t, self.r, self.own, self.forced = row, t, r, own, forced


def run(D, F, perm, beta, seed, sweep_offset=0, rep_ids=None, inst_id=0, E_best=None,
        perm_best=None, record_choices=False, record_trace=False, paranoid=False,
        tie_cap=100_000, forced=None) -> RunResult:
    """Run len(beta) sweeps on every row of ``perm`` (a copy; the input is
    left untouched).  Without ``E_best`` the best state starts from the
    initial one.  ``forced`` ([R, T, N], optional): draws of another
    evaluation of the same dynamics; the oracle adopts a forced draw only
    where its own draw is a tie and raises OracleMismatch at the first
    disagreement off a tie."""
    D, F = _i32(D), _i32(F)
    N = D.shape[0]
    p = np.array(perm, dtype=np.int32, copy=True).reshape(-1, N)
    R = p.shape[0]
    beta = np.ascontiguousarray(beta, dtype=np.float32)
    T = beta.shape[0]
    E = np.zeros(R, dtype=np.int64)
    init_best = E_best is None
    Eb = np.zeros(R, dtype=np.int64) if init_best else np.array(E_best, dtype=np.int64, copy=True)
    pb = (np.zeros((R, N), dtype=np.int32) if init_best
          else np.array(perm_best, dtype=np.int32, copy=True).reshape(R, N))
    counters = np.zeros((R, 3), dtype=np.int64)
    tie_log = np.zeros((tie_cap, 3), dtype=np.int32)
    tie_n = np.zeros(1, dtype=np.int64)
    choices = np.full((R, T, N), -1, dtype=np.int32) if record_choices else None
    trace = np.zeros((R, T), dtype=np.int64) if record_trace else None
    reps = None if rep_ids is None else np.ascontiguousarray(rep_ids, dtype=np.int32)
    fc = None
    excused = fail_at = None
    if forced is not None:
        fc = np.ascontiguousarray(forced, dtype=np.int32)
        if fc.shape != (R, T, N):
            raise ValueError(f"forced draws must have shape {(R, T, N)}, not {fc.shape}")
        excused = np.zeros(R, dtype=np.int64)
        fail_at = np.full(5, -1, dtype=np.int64)
    rc = lib().po_run(N, D, F, R, None if reps is None else reps.ctypes.data, int(inst_id), p,
                      beta, T, int(seed), int(sweep_offset), E, Eb, pb, int(init_best),
                      counters, tie_log.ctypes.data, tie_cap, tie_n.ctypes.data,
                      None if choices is None else choices.ctypes.data,
                      None if trace is None else trace.ctypes.data, int(paranoid),
                      None if fc is None else fc.ctypes.data,
                      None if excused is None else excused.ctypes.data,
                      None if fail_at is None else fail_at.ctypes.data)
    if rc == PO_EMISMATCH and fc is not None and fail_at[0] >= 0:
        raise OracleMismatch(*(int(v) for v in fail_at))
    if rc != PO_OK:
        raise RuntimeError(f"oracle run failed with status {rc}")
    return RunResult(p, E, Eb, pb, counters, tie_log[: int(tie_n[0])].copy(), choices, trace,
                     excused)


def pt_exchange(E, slot_of, since_top, timeout):
    """One parallel-tempering exchange pass over a set (Methods, "CPU-PIM
    Algorithm"); returns (slot_of, since_top, highest slot changed)."""
    E = np.ascontiguousarray(E, dtype=np.int64)
    sl = np.array(slot_of, dtype=np.int32, copy=True)
    st = np.array([since_top], dtype=np.int32)
    x = lib().po_pt_exchange(E.shape[0], E, sl, st, int(timeout))
    if x < 0:
        raise RuntimeError(f"oracle exchange failed with status {x}")
    return sl, int(st[0]), bool(x)


@dataclass
class PTResult:
    perm: np.ndarray
    E: np.ndarray
    E_best: np.ndarray
    perm_best: np.ndarray
    counters: np.ndarray          # [R, 3] totals
    slot: np.ndarray              # [R] slot of each replica in its set
    since_top: np.ndarray         # [R / L]


def run_pt(D, F, perm, ladder, n_periods, period_sweeps, timeout, seed, sweep_offset=0,
           slot=None, since_top=None, E_best=None, perm_best=None, inst_id=0,
           method="sequential") -> PTResult:
    """Parallel tempering: sets of L = len(ladder) replicas (rows of perm in
    order), n_periods periods of period_sweeps sweeps (method "sequential")
    or GPU-CUPIM iterations (method "cupim") at each replica's slot
    temperature, each followed by an exchange pass."""
    D, F = _i32(D), _i32(F)
    N = D.shape[0]
    p = np.array(perm, dtype=np.int32, copy=True).reshape(-1, N)
    R = p.shape[0]
    ladder = np.ascontiguousarray(ladder, dtype=np.float32)
    L = ladder.shape[0]
    sl = (np.tile(np.arange(L, dtype=np.int32), R // L) if slot is None
          else np.array(slot, dtype=np.int32, copy=True))
    st = np.zeros(R // L, dtype=np.int32) if since_top is None else np.array(since_top, dtype=np.int32, copy=True)
    E = np.zeros(R, dtype=np.int64)
    init_best = E_best is None
    Eb = np.zeros(R, dtype=np.int64) if init_best else np.array(E_best, dtype=np.int64, copy=True)
    pb = (np.zeros((R, N), dtype=np.int32) if init_best
          else np.array(perm_best, dtype=np.int32, copy=True).reshape(R, N))
    counters = np.zeros((R, 3), dtype=np.int64)
    rc = lib().po_run_pt(N, D, F, R, L, p, ladder, sl, st, int(n_periods), int(period_sweeps),
                         int(timeout), int(seed), int(sweep_offset), int(inst_id), E, Eb, pb,
                         int(init_best), counters, {"sequential": 0, "cupim": 1}[method])
    if rc != PO_OK:
        raise RuntimeError(f"oracle parallel tempering failed with status {rc}")
    return PTResult(p, E, Eb, pb, counters, sl, st)


def cupim_resolve(sel, dE):
    """GPU-CUPIM conflict resolution (Methods, "GPU-CUPIM Algorithm"):
    returns the boolean winner mask of the proposals r -> sel[r]."""
    sel = np.ascontiguousarray(sel, dtype=np.int32)
    dE = np.ascontiguousarray(dE, dtype=np.int64)
    win = np.zeros(sel.shape[0], dtype=np.uint8)
    n = lib().po_cupim_resolve(sel.shape[0], sel, dE, win)
    if n < 0:
        raise RuntimeError(f"oracle resolution failed with status {n}")
    return win.astype(bool)


@dataclass
class CupimResult:
    perm: np.ndarray
    E: np.ndarray
    E_best: np.ndarray
    perm_best: np.ndarray
    counters: np.ndarray          # [R, 3]: updates, accepted (winning exchanges), ties
    choices: np.ndarray | None    # [R, T, N] every draw
    won: np.ndarray | None        # [R, T, N] winner masks


def run_cupim(D, F, perm, beta, seed, sweep_offset=0, rep_ids=None, inst_id=0, E_best=None,
              perm_best=None, record=False) -> CupimResult:
    """GPU-CUPIM iterations (Results, "GPU Implementations"; Methods,
    "GPU-CUPIM Algorithm") on every row of perm; `choices` holds the draws
    and `trace` the winner masks when record is set."""
    D, F = _i32(D), _i32(F)
    N = D.shape[0]
    p = np.array(perm, dtype=np.int32, copy=True).reshape(-1, N)
    R = p.shape[0]
    beta = np.ascontiguousarray(beta, dtype=np.float32)
    T = beta.shape[0]
    ids = None if rep_ids is None else np.ascontiguousarray(rep_ids, dtype=np.int32)
    E = np.zeros(R, dtype=np.int64)
    init_best = E_best is None
    Eb = np.zeros(R, dtype=np.int64) if init_best else np.array(E_best, dtype=np.int64, copy=True)
    pb = (np.zeros((R, N), dtype=np.int32) if init_best
          else np.array(perm_best, dtype=np.int32, copy=True).reshape(R, N))
    counters = np.zeros((R, 3), dtype=np.int64)
    choices = np.full((R, T, N), -1, dtype=np.int32) if record else None
    won = np.zeros((R, T, N), dtype=np.uint8) if record else None
    rc = lib().po_run_cupim(N, D, F, R, None if ids is None else ids.ctypes.data, int(inst_id), p,
                            beta, T, int(seed), int(sweep_offset), E, Eb, pb, int(init_best),
                            counters, None if choices is None else choices.ctypes.data,
                            None if won is None else won.ctypes.data)
    if rc != PO_OK:
        raise RuntimeError(f"oracle CUPIM run failed with status {rc}")
    return CupimResult(p, E, Eb, pb, counters, choices, None if won is None else won.astype(bool))


def beta_rule(E_sum, grid, L, level_pct=40):
    """The range rule of the beta selection (Results, "Implementation";
    Methods, "CPU-PIM Algorithm") on summed trial energies, with the low
    end's level level_pct percent of the range above the minimum: returns
    (lo, hi, ladder)."""
    E_sum = np.ascontiguousarray(E_sum, dtype=np.int64)
    grid = np.ascontiguousarray(grid, dtype=np.float32)
    ladder = np.zeros(int(L), dtype=np.float32)
    lo_hi = np.zeros(2, dtype=np.int32)
    rc = lib().po_beta_rule(E_sum.shape[0], E_sum, grid, int(L), int(level_pct), ladder, lo_hi)
    if rc != PO_OK:
        raise RuntimeError(f"oracle beta rule failed with status {rc}")
    return int(lo_hi[0]), int(lo_hi[1]), ladder


@dataclass
class BetaSelection:
    E_sum: np.ndarray      # [G] summed ending energies of the trials
    E_trial: np.ndarray    # [G, R] every trial replica's ending energy
    lo: int
    hi: int
    ladder: np.ndarray     # [L]


def beta_select(D, F, perm, grid, trial_sweeps, seed, L, inst_id=0,
                level_pct=40) -> BetaSelection:
    """Beta-range selection: fixed-beta trials of trial_sweeps sweeps from
    the rows of perm at every grid value, then the range rule (low-end
    level level_pct percent of the range above the minimum) and a geometric
    ladder of L rungs."""
    D, F = _i32(D), _i32(F)
    N = D.shape[0]
    p = np.ascontiguousarray(perm, dtype=np.int32).reshape(-1, N)
    R = p.shape[0]
    grid = np.ascontiguousarray(grid, dtype=np.float32)
    G = grid.shape[0]
    E_sum = np.zeros(G, dtype=np.int64)
    E_trial = np.zeros((G, R), dtype=np.int64)
    ladder = np.zeros(int(L), dtype=np.float32)
    lo_hi = np.zeros(2, dtype=np.int32)
    rc = lib().po_beta_select(N, D, F, R, p, grid, G, int(trial_sweeps), int(seed), int(inst_id),
                              int(L), int(level_pct), E_sum, ladder.ctypes.data,
                              lo_hi.ctypes.data, E_trial.ctypes.data)
    if rc != PO_OK:
        raise RuntimeError(f"oracle beta selection failed with status {rc}")
    return BetaSelection(E_sum, E_trial, int(lo_hi[0]), int(lo_hi[1]), ladder)


def brute_min(D, F, first=-1) -> tuple[int, np.ndarray]:
    """Exhaustive minimum of Eq. 1 over all permutations (with p[0] = first
    when first >= 0)."""
    D, F = _i32(D), _i32(F)
    N = D.shape[0]
    bp = np.zeros(N, dtype=np.int32)
    e = int(lib().po_brute_min(N, D, F, int(first), bp))
    return e, bp
