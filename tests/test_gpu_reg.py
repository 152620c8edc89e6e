"""The register sweep kernel (PDIT_SWEEP_REG: G = D F[p,:] in registers,
128 < N <= 256, 8-bit D and F) against the oracle: recorded runs replayed
draw by draw (``parity.py``) at ragged and full sizes, zero and nonzero
diagonals, unsigned and signed 8-bit data, hot, cold, constant and zero
beta, an odd replica count (the second slot of the last workgroup idle),
plateau moves, resume across calls, AUTO choosing it, sweeps switching
between single updates and batches, windows of the N=256 workload's
schedule, and that workload's 512 replicas against the on-chip H kernel."""
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


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def run(ctx, D, F, perms, beta, seed, offset=0, record=True, best=None):
    R, N = perms.shape
    T = len(beta)
    p = dev(perms, torch.int32)
    ch = tr = None
    if record:
        ch = torch.full((R, T, N), -1, dtype=torch.int32, device=DEV)
        tr = torch.zeros((R, T), dtype=torch.int64, device=DEV)
        ctx.set_recording(ch, tr)
    ctx.set_sweep_offset(offset)
    ctx.run_sweeps(dev(D, torch.int32), dev(F, torch.int32), p, dev(beta, torch.float32), seed)
    Eb, pb = ctx.best()
    out = {"perm": p.cpu().numpy(), "E": ctx.energy().cpu().numpy(), "E_best": Eb.cpu().numpy(),
           "perm_best": pb.cpu().numpy(), "counters": ctx.replica_counters().cpu().numpy(),
           "choices": None if ch is None else ch.cpu().numpy(),
           "trace": None if tr is None else tr.cpu().numpy(), "plan": ctx.last_plan()}
    return out


def instance(rng, N, kind):
    if kind == "euclid":
        D = W.euclid_points(rng, N)
        F = W.sym_bernoulli_values(rng, N, 0.1, 1, 1)
    elif kind == "u8":
        D = W.sym_uniform(rng, N, 0, 255)
        F = W.sym_bernoulli_values(rng, N, 0.04, 1, 3)
    elif kind == "s8":
        D = W.sym_uniform(rng, N, -40, 40)
        F = W.sym_uniform(rng, N, -3, 3, zero_frac=0.7)
    elif kind == "diag":
        D, F = W.random_instance(rng, N, 0, 9, zero_diag=False)
        F = (F * (rng.random((N, N)) < 0.15)).astype(np.int32)
        F = np.triu(F, 1) + np.triu(F, 1).T + np.diag(np.diag(F))
    else:
        raise ValueError(kind)
    return D.astype(np.int32), F.astype(np.int32)


@pytest.mark.parametrize("N,R,T,kind,sched", [
    (129, 2, 6, "euclid", "hot"), (150, 3, 5, "u8", "hot"), (200, 4, 4, "s8", "hot"),
    (255, 3, 4, "diag", "hot"), (256, 4, 4, "euclid", "hot"), (256, 5, 30, "euclid", "cold"),
    (170, 2, 20, "u8", "cold"), (256, 2, 3, "euclid", "zero"), (230, 3, 6, "s8", "constant")])
def test_reg_matches_oracle(N, R, T, kind, sched):
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(N * 11 + T)
    D, F = instance(rng, N, kind)
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    beta = {"hot": W.beta_geometric(0.5 / s, 5.0 / s, T),
            "cold": W.beta_geometric(50.0 / s, 2000.0 / s, T),
            "zero": np.zeros(T, np.float32),
            "constant": np.full(T, 3.0 / s, np.float32)}[sched]
    say(f"reg N={N} R={R} T={T} {kind} {sched}")
    with P.Pdit(sweep="reg") as ctx:
        got = run(ctx, D, F, perms, beta, 17)
    assert got["plan"]["sweep"] == "reg"
    replay(got, D, F, perms, beta, 17, what=f"reg N={N} {kind} {sched}")
    if sched in ("hot", "zero", "constant"):
        assert got["counters"][:, 1].sum() > 0
    if sched == "zero":
        for k in range(R):
            for t in range(T):
                for r in range(N):
                    assert got["choices"][k, t, r] == (oracle.uniform24(17, r, t, k, 0) * N) >> 24


def test_reg_plateau_and_resume():
    """Two facilities with identical flows (cold replicas keep exchanging them
    at dE = 0); two calls equal one."""
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(9)
    N, R, T = 180, 3, 40
    D, F = instance(rng, N, "u8")
    F[1, :] = F[0, :]
    F[:, 1] = F[:, 0]
    F[0, 1] = F[1, 0] = 2
    F[0, 0] = F[1, 1] = 0
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    beta = W.beta_geometric(5.0 / s, 500.0 / s, T)
    with P.Pdit(sweep="reg") as ctx:
        got = run(ctx, D, F, perms, beta, 21)
    replay(got, D, F, perms, beta, 21, what="reg plateau")
    with P.Pdit(sweep="reg") as ctx:
        a = run(ctx, D, F, perms, beta[:15], 21, record=False)
        b = run(ctx, D, F, a["perm"], beta[15:], 21, offset=15, record=False)
    for key in ("perm", "E", "E_best", "perm_best"):
        assert np.array_equal(got[key], b[key]), key


@pytest.mark.parametrize("N,R", [(203, 3), (256, 2)])
def test_reg_batches_and_switches(N, R):
    """Sweeps that accept few exchanges are followed by sweeps evaluated in
    batches of updates on one state (the prefix up to the first exchange
    committed), of 12, 8 or 4 updates as the exchanges fall below 25, 49 and
    113; a schedule alternating cold and hot stretches, from an annealed
    state, then cooling from a warm one, switches between the ways several
    times and takes every batch size.  N = 203 leaves a ragged last batch in
    every sweep."""
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(N + 5)
    D, F = instance(rng, N, "euclid")
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    cold, hot = 2000.0 / s, 2.0 / s
    pre = W.beta_geometric(5.0 / s, cold, 60)
    blocks = [(cold, 4), (hot, 2), (cold, 5), (hot, 1), (cold, 3), (150.0 / s, 4),
              (300.0 / s, 4), (600.0 / s, 3)]
    beta = np.concatenate([np.full(n, b, np.float32) for b, n in blocks])
    with P.Pdit(sweep="reg") as ctx:
        a = run(ctx, D, F, perms, pre, 5, offset=500, record=False)
        start = a["perm"]
        ctx.reset()
        got = run(ctx, D, F, start, beta, 5)
    replay(got, D, F, start, beta, 5, what=f"reg switches N={N}")
    # exchanges per sweep: single updates and each batch size follow each other
    moved = (got["choices"] != np.arange(N)[None, None, :]).sum(axis=2)[:, :-1]
    for lo, hi in ((0, 24), (25, 48), (49, 112), (113, N)):
        assert ((moved >= lo) & (moved <= hi)).any(), (lo, hi, moved)


def test_reg_auto_and_refusals():
    """AUTO takes the register kernel where the data fit and the other kernels
    where they do not; a forced REG on data that do not fit is refused."""
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(4)
    D, F = instance(rng, 200, "euclid")
    perms = W.random_perms(rng, 2, 200)
    beta = np.full(2, 0.01, np.float32)
    with P.Pdit() as ctx:
        assert run(ctx, D, F, perms, beta, 3, record=False)["plan"]["sweep"] == "reg"
    for N, hi in ((200, 300), (100, 50), (300, 9)):
        D2, F2 = W.random_instance(rng, N, 0, hi)
        p2 = W.random_perms(rng, 2, N)
        with P.Pdit() as ctx:
            assert run(ctx, D2, F2, p2, beta, 3, record=False)["plan"]["sweep"] != "reg"
        with P.Pdit(sweep="reg") as ctx:
            with pytest.raises(P.PditError) as e:
                run(ctx, D2, F2, p2, beta, 3, record=False)
            assert e.value.status == "PDIT_EOVERFLOW"


@pytest.mark.parametrize("where", ["start", "middle", "cooling", "cool", "end"])
def test_reg_n256_workload_windows(where):
    """The N=256 workload: 8 of its 512 replicas (rows 0, 73, ..., 511 of the
    full batch, with their own Philox replica indices) over a window of 200
    sweeps at the start, the middle, two cooling points (batches of 4 and 8
    updates) and the cold end (batches of 12) of its 10^5-sweep schedule,
    each window started from the GPU's own state after a strided pass over
    the schedule before it; the window replayed draw by draw."""
    from paper_2605_24408_amd import pdit as P
    inst = W.config_n256()
    rows = [0, 73, 146, 219, 292, 365, 438, 511]
    start = {"start": 0, "middle": 50_000, "cooling": 65_000, "cool": 72_500,
             "end": 99_800}[where]
    win = 200
    # the full batch, so the sampled rows keep their replica indices
    perms = inst.perms.copy()
    with P.Pdit() as ctx:
        if start:
            # reach the window's temperature: every 100th beta of the schedule
            # up to the window, a cheap anneal on the GPU's own trajectory
            pre = inst.beta[:start:100].copy()
            a = run(ctx, inst.D, inst.F, perms, pre, W.PHILOX_SEED, offset=10**6, record=False)
            perms = a["perm"]
        say(f"n256 window at {start}")
        ctx.reset()
        got = run(ctx, inst.D, inst.F, perms, inst.beta[start:start + win], W.PHILOX_SEED,
                  offset=start)
    assert got["plan"]["sweep"] == "reg"
    parts = replay(got, inst.D, inst.F, perms[rows], inst.beta[start:start + win],
                   W.PHILOX_SEED, offset=start, rows=rows, threads=8,
                   what=f"n256 window at {start}")
    acc = sum(int(p.counters[0][1]) for p in parts)
    say(f"window at {start}: acceptance {acc / (len(rows) * 256 * win):.4f}")


def test_reg_equals_h_kernel_on_all_replicas():
    """Every exact kernel takes the same integer draws, so the register kernel
    and the class-256 on-chip H kernel must end in identical states on all
    512 replicas of the N=256 workload over a strided pass of its schedule
    (every 50th beta up to sweep 75 000: hot sweeps one update at a time,
    then batches).  Unlike the sampled oracle replays this covers every
    replica and both replica slots of every workgroup, so a race between the
    waves of one replica shows up as a difference."""
    from paper_2605_24408_amd import pdit as P
    inst = W.config_n256()
    beta = inst.beta[:75_000:50].copy()
    outs = {}
    for sweep in ("reg", "fast"):
        with P.Pdit(sweep=sweep) as ctx:
            outs[sweep] = run(ctx, inst.D, inst.F, inst.perms, beta, W.PHILOX_SEED, record=False)
            assert outs[sweep]["plan"]["sweep"] == sweep
    a, b = outs["reg"], outs["fast"]
    for key in ("perm", "E", "E_best", "perm_best"):
        bad = np.nonzero((a[key] != b[key]).reshape(len(a[key]), -1).any(axis=1))[0]
        assert bad.size == 0, f"{key} differs in replicas {bad[:16]} ({bad.size} of 512)"
    assert np.array_equal(a["counters"][:, :2], b["counters"][:, :2])
    say(f"reg = fast on 512 replicas x {len(beta)} sweeps; accepted "
        f"{int(a['counters'][:, 1].sum())}")
