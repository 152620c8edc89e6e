"""GPU-CUPIM on the GPU (pdit_run_cupim) against the oracle's run_cupim:
every size class, zero and nonzero diagonals, hot and cold schedules,
resume across calls, the N=64 benchmark instance at full size with sampled
replicas, error paths."""
import numpy as np
import pytest
import torch

import oracle
from paper_2605_24408_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda", 0)


def say(msg):
    print(msg, flush=True)


def dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype)


def gpu_cupim(ctx, D, F, perms, beta, seed):
    p = dev(perms, torch.int32)
    ctx.run_cupim(dev(D, torch.int32), dev(F, torch.int32), p, dev(beta, torch.float32), seed)
    Eb, pb = ctx.best()
    return {"perm": p.cpu().numpy(), "E": ctx.energy().cpu().numpy(), "E_best": Eb.cpu().numpy(),
            "perm_best": pb.cpu().numpy(), "counters": ctx.replica_counters().cpu().numpy()}


def compare(got, ref):
    R = ref.perm.shape[0]
    bad = [k for k in range(R)
           if not (np.array_equal(got["perm"][k], ref.perm[k]) and got["E"][k] == ref.E[k]
                   and got["E_best"][k] == ref.E_best[k]
                   and np.array_equal(got["perm_best"][k], ref.perm_best[k])
                   and np.array_equal(got["counters"][k], ref.counters[k]))]
    for k in bad:
        assert ref.counters[k][2] > 0, (
            f"replica {k} differs from the oracle without a counted tie: E {got['E'][k]} vs "
            f"{ref.E[k]}, accepted {got['counters'][k][1]} vs {ref.counters[k][1]}")
    return bad


@pytest.mark.parametrize("N,R,kind,sched", [
    (2, 6, "uniform", "hot"), (5, 4, "diag", "hot"), (12, 4, "grid", "anneal"),
    (16, 4, "uniform", "anneal"), (33, 3, "uniform", "hot"), (40, 3, "diag", "anneal"),
    (64, 3, "uniform", "anneal"), (64, 2, "uniform", "hot"), (100, 2, "diag", "anneal"),
    (128, 2, "uniform", "anneal")])
def test_cupim_matches_oracle(N, R, kind, sched):
    from paper_2605_24408_amd import pdit as P
    say(f"cupim N={N} R={R} kind={kind} sched={sched}")
    rng = np.random.default_rng(N * 7 + R)
    if kind == "grid":
        inst = W.config_n12(R=R, T=1)
        D, F = inst.D, inst.F
    else:
        D, F = W.random_instance(rng, N, 0, 99 if N > 10 else 9, zero_diag=(kind != "diag"))
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    T = 40
    beta = (np.full(T, 0.3 / s, np.float32) if sched == "hot"
            else W.beta_geometric(0.2 / s, 50.0 / s, T))
    ref = oracle.run_cupim(D, F, perms, beta, 13)
    with P.Pdit() as ctx:
        got = gpu_cupim(ctx, D, F, perms, beta, 13)
        plan = ctx.last_plan()
    assert plan["size_class"] >= N
    bad = compare(got, ref)
    assert len(bad) < R
    assert ref.counters[:, 1].sum() > 0


def test_cupim_resume_equals_single_call():
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(2)
    N, R = 48, 4
    D, F = W.random_instance(rng, N, 0, 60)
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    beta = W.beta_geometric(0.2 / s, 20.0 / s, 50)
    with P.Pdit() as ctx:
        one = gpu_cupim(ctx, D, F, perms, beta, 4)
    with P.Pdit() as ctx:
        a = gpu_cupim(ctx, D, F, perms, beta[:20], 4)
        b = gpu_cupim(ctx, D, F, a["perm"], beta[20:], 4)
    for f in ("perm", "E", "E_best", "perm_best"):
        assert np.array_equal(one[f], b[f]), f


def test_cupim_full_size_sampled():
    """The N=64 benchmark instance, 1024 replicas x 300 iterations of its
    schedule in one launch: sampled replicas rerun on the oracle, every
    replica's E = Eq. 1 of its permutation and E_best = Eq. 1 of perm_best."""
    from paper_2605_24408_amd import pdit as P
    inst = W.config_n64()
    T = 300
    beta = inst.beta[:T]
    with P.Pdit() as ctx:
        got = gpu_cupim(ctx, inst.D, inst.F, inst.perms, beta, W.PHILOX_SEED)
    Di, Fi = inst.D.astype(np.int64), inst.F.astype(np.int64)
    energy = lambda p: int((Di * Fi[np.ix_(p, p)]).sum())
    for k in range(0, inst.R, 97):
        assert sorted(got["perm"][k]) == list(range(64))
        assert got["E"][k] == energy(got["perm"][k])
        assert got["E_best"][k] == energy(got["perm_best"][k]) <= energy(inst.perms[k])
    assert np.all(got["counters"][:, 0] == 64 * T)
    for k in (0, 511, 1023):
        ref = oracle.run_cupim(inst.D, inst.F, inst.perms[k:k + 1], beta, W.PHILOX_SEED,
                               rep_ids=[k])
        if ref.counters[0][2] == 0:
            assert np.array_equal(got["perm"][k], ref.perm[0]), k
            assert got["E_best"][k] == ref.E_best[0], k
            assert got["counters"][k][1] == ref.counters[0][1], k


def test_cupim_error_paths():
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(1)
    with P.Pdit() as ctx:
        D, F = W.random_instance(rng, 130, 0, 9)
        with pytest.raises(P.PditError) as e:
            gpu_cupim(ctx, D, F, W.random_perms(rng, 2, 130), np.ones(2, np.float32), 1)
        assert e.value.status == "PDIT_EOVERFLOW"
        D, F = W.random_instance(rng, 20, 0, 200)
        with pytest.raises(P.PditError) as e:
            gpu_cupim(ctx, D, F, W.random_perms(rng, 2, 20), np.ones(2, np.float32), 1)
        assert e.value.status == "PDIT_EOVERFLOW"
        D, F = W.random_instance(rng, 20, 0, 9)
        with pytest.raises(P.PditError) as e:
            gpu_cupim(ctx, D, F, W.random_perms(rng, 2, 20), np.array([0.1, -1.0], np.float32), 1)
        assert e.value.status == "PDIT_EBETA"
        # zero iterations: energies of the given permutations, nothing moves
        perms = W.random_perms(rng, 3, 20)
        got = gpu_cupim(ctx, D, F, perms, np.zeros(0, np.float32), 1)
        assert np.array_equal(got["perm"], perms)
        assert got["counters"].sum() == 0
