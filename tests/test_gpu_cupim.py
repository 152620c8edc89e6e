"""GPU-CUPIM on the GPU (pdit_run_cupim) against the oracle's run_cupim:
every size class, zero and nonzero diagonals, hot and cold schedules,
resume across calls, the N=64 benchmark instance at full size with sampled
replicas, error paths.  The launches do not record their draws, so parity
is checked iteration by iteration (``parity.py``): after every iteration
each replica must equal the oracle's iteration from the same state, unless
the oracle counted a tie in that replica's iteration; the oracle is then
re-synced to the GPU's state."""
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


def cupim_chunked(P, D, F, perms, beta, seed, chunk=1, rows=None, what="cupim"):
    """The GPU run in calls of ``chunk`` iterations; after each call the
    replicas ``rows`` (default all) must equal the oracle's run of the same
    iterations from the GPU's previous state, unless the oracle counted a tie
    for that replica in them.  Returns the final GPU state and the plan."""
    R = perms.shape[0]
    rows = list(range(R)) if rows is None else list(rows)
    T = len(beta)
    state = {"perm": perms[rows], "E_best": None, "perm_best": None}
    resync = 0
    with P.Pdit() as ctx:
        p = dev(perms, torch.int32)
        Dd, Fd = dev(D, torch.int32), dev(F, torch.int32)
        done = 0
        while done < T:
            k = min(chunk, T - done)
            ctx.run_cupim(Dd, Fd, p, dev(beta[done:done + k], torch.float32), seed)
            Eb, pb = ctx.best()
            got = {"perm": p.cpu().numpy(), "E": ctx.energy().cpu().numpy(),
                   "E_best": Eb.cpu().numpy(), "perm_best": pb.cpu().numpy(),
                   "counters": ctx.replica_counters().cpu().numpy()}
            ref = oracle.run_cupim(D, F, state["perm"], beta[done:done + k], seed,
                                   sweep_offset=done, rep_ids=rows, E_best=state["E_best"],
                                   perm_best=state["perm_best"])
            for i, r in enumerate(rows):
                same = (np.array_equal(got["perm"][r], ref.perm[i]) and got["E"][r] == ref.E[i]
                        and got["E_best"][r] == ref.E_best[i]
                        and np.array_equal(got["perm_best"][r], ref.perm_best[i])
                        and np.array_equal(got["counters"][r][:2], ref.counters[i][:2]))
                if not same:
                    assert ref.counters[i][2] > 0, (
                        f"{what}: iterations {done}..{done + k}, replica {r} differs from the "
                        f"oracle with no oracle tie")
                    resync += 1
            state = {"perm": got["perm"][rows], "E_best": got["E_best"][rows],
                     "perm_best": got["perm_best"][rows]}
            done += k
        plan = ctx.last_plan()
    say(f"{what}: {T} iterations in chunks of {chunk}, {resync} re-syncs at oracle ties")
    assert resync <= max(1, len(rows) * T // (10 * chunk))
    return got, plan


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
    got, plan = cupim_chunked(P, D, F, perms, beta, 13, what=f"cupim N={N} {sched}")
    assert plan["size_class"] >= N
    assert got["counters"][:, 1].sum() > 0


@pytest.mark.parametrize("N,R,hi,zero_diag,sched", [
    (150, 2, 99, True, "anneal"), (200, 2, 60, False, "hot"), (256, 2, 1000, True, "anneal"),
    (64, 3, 5000, True, "anneal"), (300, 1, 300, False, "anneal")])
def test_cupim_large_matches_oracle(N, R, hi, zero_diag, sched):
    """Beyond the on-chip kernel (N > 128 or entries beyond 8 bits): the
    snapshot in device memory, refreshed by the H recompute, iteration by
    iteration against the oracle."""
    from paper_2605_24408_amd import pdit as P
    say(f"cupim large N={N} R={R} hi={hi} zero_diag={zero_diag} {sched}")
    rng = np.random.default_rng(N * 3 + hi)
    D, F = W.random_instance(rng, N, 0, hi, zero_diag=zero_diag)
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    T = 30
    beta = (np.full(T, 0.3 / s, np.float32) if sched == "hot"
            else W.beta_geometric(0.2 / s, 50.0 / s, T))
    got, plan = cupim_chunked(P, D, F, perms, beta, 13, what=f"cupim large N={N}")
    assert plan["sweep"] == "large"
    assert got["counters"][:, 1].sum() > 0
    Di, Fi = D.astype(np.int64), F.astype(np.int64)
    for k in range(R):
        assert got["E"][k] == int((Di * Fi[np.ix_(got["perm"][k], got["perm"][k])]).sum())


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
    schedule in one launch: every replica's E = Eq. 1 of its permutation and
    E_best = Eq. 1 of perm_best; the same batch in calls of 30 iterations
    ends in the same state, with replicas 0, 511 and 1023 checked against
    the oracle after every call."""
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
    part, _ = cupim_chunked(P, inst.D, inst.F, inst.perms, beta, W.PHILOX_SEED, chunk=30,
                            rows=[0, 511, 1023], what="cupim n64 full size")
    for key in ("perm", "E", "E_best", "perm_best"):
        assert np.array_equal(part[key], got[key]), key


def test_cupim_n256_workload_sampled():
    """The N=256 workload (distances to 141: beyond the on-chip kernel) at its
    512 replicas for the first 20 iterations of its schedule: every sampled
    replica's E equals Eq. 1, and replicas 0, 255 and 511 equal the oracle
    after every iteration."""
    from paper_2605_24408_amd import pdit as P
    inst = W.config_n256()
    beta = inst.beta[:20]
    got, plan = cupim_chunked(P, inst.D, inst.F, inst.perms, beta, W.PHILOX_SEED,
                              rows=[0, 255, 511], what="cupim n256 full size")
    assert plan["sweep"] == "large"
    Di, Fi = inst.D.astype(np.int64), inst.F.astype(np.int64)
    for k in range(0, inst.R, 73):
        assert got["E"][k] == int((Di * Fi[np.ix_(got["perm"][k], got["perm"][k])]).sum())
    assert np.all(got["counters"][:, 0] == 256)   # the last call's one iteration


def test_cupim_error_paths():
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(1)
    with P.Pdit() as ctx:
        # snapshot energy changes that do not pack into the 64-bit proposal key
        D, F = W.random_instance(rng, 20, 0, 10**8)
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
