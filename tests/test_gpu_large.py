"""GPU parity of the sweep kernel that stores no H (pdit_run_sweeps with
PDIT_SWEEP_LARGE, and AUTO where no on-chip class fits): every variant of its
products (int16 or int32 copies of D and F, int32 partial sums of 24-bit
products or int64 products), int32 and int64 initial H, ragged sizes from 2
to 512, against the CPU oracle on the same seeded inputs.  Recorded runs
are replayed draw by draw on the oracle (``parity.py``): a draw may differ
only where the oracle flags a tie, and energies, permutations, best states,
counters and energy traces must then be identical."""
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2605_24408_amd import workloads as W
from parity import replay

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    from paper_2605_24408_amd import pdit
    return pdit


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).to(DEV)


def run_large(P, D, F, perms, beta, seed, sweep="large", record=True, offset=0, ctx=None):
    own = ctx is None
    if own:
        ctx = P.Pdit(sweep=sweep)
    Dd, Fd = dev(D, torch.int32), dev(F, torch.int32)
    perm = dev(perms, torch.int32)
    b = dev(np.asarray(beta, np.float32), torch.float32)
    R, N = perm.shape
    T = b.numel()
    ch = tr = None
    if record:
        ch = torch.full((R, T, N), -1, dtype=torch.int32, device=DEV)
        tr = torch.zeros((R, T), dtype=torch.int64, device=DEV)
        ctx.set_recording(ch, tr)
    ctx.set_sweep_offset(offset)
    ctx.run_sweeps(Dd, Fd, perm, b, seed)
    E = ctx.energy()
    Eb, pb = ctx.best()
    cnt = ctx.replica_counters()
    torch.cuda.synchronize()
    out = dict(perm=perm.cpu().numpy(), E=E.cpu().numpy(), E_best=Eb.cpu().numpy(),
               perm_best=pb.cpu().numpy(), counters=cnt.cpu().numpy(),
               choices=None if ch is None else ch.cpu().numpy(),
               trace=None if tr is None else tr.cpu().numpy(), plan=ctx.last_plan())
    if own:
        ctx.close()
    return out


def instance(rng, N, dmax, fmax, zero_diag=True):
    D = W.sym_uniform(rng, N, 0, dmax).astype(np.int64)
    F = W.sym_uniform(rng, N, 0, fmax).astype(np.int64)
    if not zero_diag:
        D[np.diag_indices(N)] = rng.integers(0, dmax + 1, size=N)
        F[np.diag_indices(N)] = rng.integers(0, fmax + 1, size=N)
    # the maxima pick the copy layout: make sure they occur
    D[0, 1] = D[1, 0] = max(D[0, 1], dmax * (D.max() < dmax))
    F[0, 1] = F[1, 0] = max(F[0, 1], fmax * (F.max() < fmax))
    return D.astype(np.int32), F.astype(np.int32)


# (N, R, T, max|D|, max|F|, zero diagonal, hot): the values pick the variant --
# int8 plane copies and MFMA products (eight locations per pass) when both
# maxima are <= 16383, int16 copies (three per pass) up to 32767, int32
# partial sums when 16 max|D| max|F| < 2^31, int64 H when the bound on |H|
# exceeds 2^31 - 1
CASES = [
    (2, 6, 40, 9, 9, True, True),            # int16, narrow, H int32; the smallest instance
    (7, 8, 30, 60, 60, False, True),         # nonzero diagonals
    (33, 5, 12, 60, 60, True, False),        # one wave, cold
    (64, 4, 8, 99, 99, True, True),          # exactly one wave
    (65, 4, 8, 99, 99, False, True),         # two waves, one lane of the second
    (130, 3, 4, 10_000, 10_000, True, True),   # int16, narrow, H int64
    (150, 3, 4, 30_000, 30_000, True, True),   # int16, int64 products
    (40, 4, 10, 20_000, 20_000, True, True),   # int16 pairs, N = 1 mod 3
    (259, 2, 2, 20_000, 20_000, False, True),  # int16 pairs, ragged, nonzero diagonals
    (100, 3, 5, 200_000, 600, True, True),     # int32 copies, narrow
    (90, 3, 5, 2_000_000, 5_000, False, True),  # int32 copies, int64 products, H int64
    (257, 2, 2, 10_000, 10_000, True, True),   # ragged: 5 waves, one lane of the last
    (300, 2, 2, 99, 99, True, True),
    (512, 2, 2, 10_000, 10_000, True, True),   # the largest instance
    (97, 3, 6, 16_383, 16_383, True, True),    # planes at their largest values
    (98, 3, 6, 16_384, 16_384, True, True),    # int16 pairs from here: a plane's hi byte would be 128
]


@pytest.mark.parametrize("N,R,T,dmax,fmax,zd,hot", CASES)
def test_large_trajectories(P, N, R, T, dmax, fmax, zd, hot):
    rng = np.random.default_rng(7000 + N + dmax % 97)
    D, F = instance(rng, N, dmax, fmax, zd)
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    beta = W.beta_geometric((0.05 if hot else 2.0) / s, 50.0 / s, T)
    say(f"large trajectory N={N} R={R} T={T} max|D|={dmax} max|F|={fmax}")
    got = run_large(P, D, F, perms, beta, 11)
    assert got["plan"]["sweep"] == "large"
    replay(got, D, F, perms, beta, 11, what=f"large N={N}")
    assert got["counters"][:, 1].sum() > 0
    # a single launch serves w locations per pass over the copies (8 on the
    # int8 planes, 3 on the int16 pairs): the corrections after an accepted
    # exchange whose partner is a later location of the same pass, or one of
    # the next pass, are exercised
    vmax = max(dmax, fmax)
    w = 8 if vmax <= 16_383 else 3 if vmax <= 32_767 else 0
    if hot and w and N >= 2 * w:
        r = np.arange(N)[None, None, :]
        s = got["choices"]
        r0 = (r // w) * w
        assert ((s > r) & (s < r0 + w)).sum() > 0
        assert ((s >= r0 + w) & (s < r0 + 2 * w)).sum() > 0


@pytest.mark.parametrize("N,vmax", [(70, 5_000), (71, 16_383), (45, 30_000)])
def test_large_signed_values(P, N, vmax):
    """Negative entries (D and F symmetric, uniform in [-vmax, vmax]): the
    int8 planes split x = 128 hi + lo with hi negative, the int16 pairs
    carry the sign in each half."""
    rng = np.random.default_rng(900 + N)
    D = W.sym_uniform(rng, N, -vmax, vmax).astype(np.int32)
    F = W.sym_uniform(rng, N, -vmax, vmax).astype(np.int32)
    perms = W.random_perms(rng, 3, N)
    s = W.energy_scale(D, F)
    beta = W.beta_geometric(0.05 / s, 50.0 / s, 6)
    say(f"large signed N={N} max={vmax}")
    got = run_large(P, D, F, perms, beta, 13)
    assert got["plan"]["sweep"] == "large"
    replay(got, D, F, perms, beta, 13, what=f"large signed N={N}")
    assert got["counters"][:, 1].sum() > 0


def test_auto_picks_large(P):
    """AUTO runs the kernel without a stored H where no on-chip class fits
    (N > 256, or values beyond the fast kernel's), with the same results."""
    rng = np.random.default_rng(5)
    for N, dmax in ((280, 50), (120, 100_000)):
        D, F = instance(rng, N, dmax, 40)
        perms = W.random_perms(rng, 2, N)
        s = W.energy_scale(D, F)
        beta = W.beta_geometric(0.2 / s, 20.0 / s, 2)
        say(f"auto N={N} max|D|={dmax}")
        got = run_large(P, D, F, perms, beta, 3, sweep="auto")
        assert got["plan"]["sweep"] == "large"
        replay(got, D, F, perms, beta, 3, what=f"auto N={N}")


def test_resume_matches_one_call(P):
    """Two calls of T sweeps (the second from the first's state and sweep
    offset) give what one call of 2T sweeps gives."""
    rng = np.random.default_rng(21)
    N, R, T = 260, 3, 2
    D, F = instance(rng, N, 500, 500)
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    beta = W.beta_geometric(0.1 / s, 10.0 / s, 2 * T)
    say("large resume")
    one = run_large(P, D, F, perms, beta, 9, record=False)
    with P.Pdit(sweep="large") as ctx:
        perm = dev(perms, torch.int32)
        Dd, Fd = dev(D, torch.int32), dev(F, torch.int32)
        ctx.run_sweeps(Dd, Fd, perm, dev(beta[:T], torch.float32), 9)
        ctx.run_sweeps(Dd, Fd, perm, dev(beta[T:], torch.float32), 9)
        E = ctx.energy().cpu().numpy()
        Eb, pb = ctx.best()
        torch.cuda.synchronize()
        assert np.array_equal(perm.cpu().numpy(), one["perm"])
        assert np.array_equal(E, one["E"])
        assert np.array_equal(Eb.cpu().numpy(), one["E_best"])
        assert np.array_equal(pb.cpu().numpy(), one["perm_best"])


def test_n512_workload_sampled(P):
    """The N=512 workload (D, F uniform in [0, 10^4] with 20% zeros) at its
    full replica count, 256, in the launch the benchmark times, for the
    first sweeps of its schedule, then again with every draw recorded
    (identical results): replicas 0, 97 and 255 replayed draw by draw on the
    oracle (same Philox replica indices), and every replica's energy equals
    the energy of its final permutation."""
    inst = W.config_n512()
    T = 2
    beta = inst.beta[:T]
    say("n512 sampled")
    got = run_large(P, inst.D, inst.F, inst.perms, beta, W.PHILOX_SEED, sweep="auto",
                    record=False)
    assert got["plan"]["sweep"] == "large"
    rec = run_large(P, inst.D, inst.F, inst.perms, beta, W.PHILOX_SEED, sweep="auto")
    for key in ("perm", "E", "E_best", "perm_best", "counters"):
        assert np.array_equal(got[key], rec[key]), key
    rows = [0, 97, 255]
    replay(rec, inst.D, inst.F, inst.perms[rows], beta, W.PHILOX_SEED, rows=rows, threads=3,
           what="n512 workload")
    for k in range(0, 256, 15):
        assert got["E"][k] == oracle.energy(inst.D, inst.F, got["perm"][k])
        assert got["E_best"][k] == oracle.energy(inst.D, inst.F, got["perm_best"][k])
    assert (got["counters"][:, 0] == 512 * T).all()


@pytest.mark.parametrize("where", ["start", "warm", "middle", "end"])
def test_n512_workload_windows(P, where):
    """The N=512 workload at its full replica count (256, so the sampled rows
    keep their Philox replica indices) over windows of its 2x10^4-sweep
    schedule: the first 100 sweeps, and 200 sweeps at sweep 6000 (where the
    acceptance falls, about 0.27), at the middle and at the cold end, each started from the GPU's own state after a strided pass
    over the schedule before it (every 100th beta) and at the window's own
    sweep offset; 8 replicas replayed draw by draw on the oracle from the
    same state."""
    inst = W.config_n512()
    rows = [0, 37, 73, 110, 146, 183, 219, 255]
    start, win = {"start": (0, 100), "warm": (6_000, 200), "middle": (10_000, 200),
                  "end": (19_800, 200)}[where]
    perms = inst.perms.copy()
    if start:
        pre = inst.beta[:start:100].copy()
        perms = run_large(P, inst.D, inst.F, perms, pre, W.PHILOX_SEED, sweep="auto",
                          record=False, offset=10**6)["perm"]
    say(f"n512 window at {start}")
    beta = inst.beta[start:start + win]
    got = run_large(P, inst.D, inst.F, perms, beta, W.PHILOX_SEED, sweep="auto", offset=start)
    assert got["plan"]["sweep"] == "large"
    parts = replay(got, inst.D, inst.F, perms[rows], beta, W.PHILOX_SEED, offset=start,
                   rows=rows, threads=8, what=f"n512 window at {start}")
    acc = sum(int(p.counters[0][1]) for p in parts)
    say(f"n512 window at {start}: acceptance {acc / (len(rows) * 512 * win):.4f}")
    for k in range(0, 256, 51):
        assert got["E"][k] == oracle.energy(inst.D, inst.F, got["perm"][k])
