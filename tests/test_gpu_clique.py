"""The clique-flow sweep (PDIT_SWEEP_CLIQUE) against the oracle's general
sweep: same dynamics, so every recorded draw is replayed on the oracle
(``parity.py``: a draw may differ only at an oracle tie) and energies, best
states and counters must agree.  Sizes on both sides of 128 (forced and automatic), up to N = 512;
random and prefix cliques; a grid-distance tai256c stand-in at full size
with sampled replicas; plan selection and error paths."""
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


def run_gpu(ctx, D, F, perms, beta, seed, record=False):
    p = dev(perms, torch.int32)
    R, N = perms.shape
    T = len(beta)
    ch = tr = None
    if record:
        ch = torch.full((R, T, N), -1, dtype=torch.int32, device=DEV)
        tr = torch.zeros((R, T), dtype=torch.int64, device=DEV)
        ctx.set_recording(ch, tr)
    ctx.run_sweeps(dev(D, torch.int32), dev(F, torch.int32), p, dev(beta, torch.float32), seed)
    Eb, pb = ctx.best()
    return {"perm": p.cpu().numpy(), "E": ctx.energy().cpu().numpy(), "E_best": Eb.cpu().numpy(),
            "perm_best": pb.cpu().numpy(), "counters": ctx.replica_counters().cpu().numpy(),
            "choices": None if ch is None else ch.cpu().numpy(),
            "trace": None if tr is None else tr.cpu().numpy(), "plan": ctx.last_plan()}


def clique_instance(rng, N, m, kind):
    D = W.grid_manhattan(N, 16) if kind == "grid" else W.sym_uniform(rng, N, 0, 60)
    members = np.arange(m) if kind == "grid" else rng.permutation(N)[:m]
    return D, W.clique_flows(N, members)


@pytest.mark.parametrize("N,m,R,T,kind,sweep", [
    (20, 7, 4, 30, "uniform", "clique"), (64, 30, 3, 20, "grid", "clique"),
    (100, 1, 2, 10, "uniform", "clique"), (130, 50, 2, 12, "uniform", "auto"),
    (200, 199, 2, 8, "uniform", "auto"), (256, 92, 2, 8, "grid", "auto"),
    (300, 120, 2, 5, "uniform", "auto"), (512, 200, 1, 3, "uniform", "auto")])
def test_clique_matches_oracle(N, m, R, T, kind, sweep):
    from paper_2605_24408_amd import pdit as P
    say(f"clique N={N} m={m} R={R} T={T} kind={kind} sweep={sweep}")
    rng = np.random.default_rng(N + m)
    D, F = clique_instance(rng, N, m, kind)
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    beta = W.beta_geometric(0.5 / s, 200.0 / s, T)
    with P.Pdit(sweep=sweep) as ctx:
        got = run_gpu(ctx, D, F, perms, beta, 9, record=True)
    assert got["plan"]["sweep"] == "clique"
    replay(got, D, F, perms, beta, 9, what=f"clique N={N} m={m}")
    assert got["counters"][:, 1].sum() > 0


def test_clique_resume_and_auto_plan():
    """Two calls equal one; N <= 128 keeps the table kernel under AUTO, and
    FAST keeps the general kernel, with the same results."""
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(5)
    N = 160
    D, F = clique_instance(rng, N, 60, "uniform")
    perms = W.random_perms(rng, 3, N)
    s = W.energy_scale(D, F)
    beta = W.beta_geometric(1.0 / s, 100.0 / s, 10)
    with P.Pdit() as ctx:
        one = run_gpu(ctx, D, F, perms, beta, 2)
    with P.Pdit() as ctx:
        a = run_gpu(ctx, D, F, perms, beta[:4], 2)
        b = run_gpu(ctx, D, F, a["perm"], beta[4:], 2)
    for f in ("perm", "E", "E_best", "perm_best"):
        assert np.array_equal(one[f], b[f]), f
    with P.Pdit(sweep="fast") as ctx:
        gen = run_gpu(ctx, D, F, perms, beta, 2)
    assert gen["plan"]["sweep"] == "fast" and one["plan"]["sweep"] == "clique"
    for f in ("perm", "E", "E_best", "perm_best", "counters"):
        assert np.array_equal(one[f], gen[f]), f
    D2, F2 = clique_instance(rng, 100, 40, "uniform")
    with P.Pdit() as ctx:
        got = run_gpu(ctx, D2, F2, W.random_perms(rng, 2, 100), beta[:2], 2)
    assert got["plan"]["sweep"] == "fast"


def test_clique_full_size_sampled():
    """The N=256 tai256c stand-in (16 x 16 grid distances, clique of 92),
    512 replicas x 200 sweeps of its schedule, then again with every draw
    recorded (identical results): replicas 0 and 300 replayed draw by draw
    on the oracle; E = Eq. 1 of every sampled permutation and best."""
    from paper_2605_24408_amd import pdit as P
    inst = W.config_clique256()
    T = 200
    beta = inst.beta[:T]
    with P.Pdit() as ctx:
        got = run_gpu(ctx, inst.D, inst.F, inst.perms, beta, W.PHILOX_SEED)
    assert got["plan"]["sweep"] == "clique"
    Di, Fi = inst.D.astype(np.int64), inst.F.astype(np.int64)
    energy = lambda p: int((Di * Fi[np.ix_(p, p)]).sum())
    for k in range(0, inst.R, 51):
        assert sorted(got["perm"][k]) == list(range(256))
        assert got["E"][k] == energy(got["perm"][k])
        assert got["E_best"][k] == energy(got["perm_best"][k])
    with P.Pdit() as ctx:
        rec = run_gpu(ctx, inst.D, inst.F, inst.perms, beta, W.PHILOX_SEED, record=True)
    for key in ("perm", "E", "E_best", "perm_best", "counters"):
        assert np.array_equal(got[key], rec[key]), key
    rows = [0, 300]
    replay(rec, inst.D, inst.F, inst.perms[rows], beta, W.PHILOX_SEED, rows=rows, threads=2,
           what="clique stand-in")


def test_clique_error_paths():
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(7)
    N = 150
    D, F = clique_instance(rng, N, 40, "uniform")
    perms = W.random_perms(rng, 2, N)
    beta = np.full(2, 0.01, np.float32)
    bad_F = F.copy()
    bad_F[3, 4] = bad_F[4, 3] = 2  # not 0/1
    bad_D = D.copy()
    bad_D[5, 5] = 1  # nonzero diagonal
    with P.Pdit(sweep="clique") as ctx:
        for Dx, Fx in ((D, bad_F), (bad_D, F)):
            with pytest.raises(P.PditError) as e:
                run_gpu(ctx, Dx, Fx, perms, beta, 1)
            assert e.value.status == "PDIT_EINVAL"
    # AUTO falls back to the general kernels on such data, with the same results
    with P.Pdit() as ctx:
        got = run_gpu(ctx, D, bad_F, perms, beta, 1)
    assert got["plan"]["sweep"] != "clique"
    with P.Pdit(sweep="clique") as ctx:
        with pytest.raises(P.PditError) as e:
            ctx.run_pt(dev(D, torch.int32), dev(F, torch.int32), dev(perms, torch.int32),
                       dev(np.array([0.1, 0.2], np.float32), torch.float32),
                       dev(np.array([0, 1]), torch.int32), dev(np.zeros(1), torch.int32), 1, 1, 5, 1)
        assert e.value.status == "PDIT_EINVAL"
