"""Beta-range selection on the GPU (pdit_beta_select) against the oracle's
beta_select: every trial replica's ending energy, the summed energies, the
chosen range and the ladder, on each sweep kernel; the ladder feeding a
parallel-tempering run; error paths."""
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


def gpu_select(ctx, D, F, perms, grid, trials, seed, L):
    Dd, Fd, pd = dev(D, torch.int32), dev(F, torch.int32), dev(perms, torch.int32)
    E_sum, ladder, rng = ctx.beta_select(Dd, Fd, pd, dev(grid, torch.float32), trials, seed, L)
    out = {"E_sum": E_sum.cpu().numpy(), "ladder": ladder.cpu().numpy(),
           "range": tuple(int(x) for x in rng.cpu().numpy()), "E": ctx.energy().cpu().numpy(),
           "counters": ctx.replica_counters().cpu().numpy(), "perm_after": pd.cpu().numpy()}
    return out


def tied_rows(D, F, perms, grid, trials, seed):
    """Trial replicas in which the oracle counts a tie."""
    R = perms.shape[0]
    rows = set()
    for g, b in enumerate(grid):
        ref = oracle.run(D, F, perms, np.full(trials, b, np.float32), seed,
                         rep_ids=[g * R + k for k in range(R)])
        rows |= {g * R + k for k in range(R) if ref.counters[k][2] > 0}
    return rows


@pytest.mark.parametrize("N,R,G,kind,sweep", [
    (12, 6, 10, "grid", "auto"), (40, 4, 12, "uniform", "auto"), (64, 4, 16, "uniform", "auto"),
    (100, 3, 8, "diag", "auto"), (140, 3, 8, "uniform", "auto"), (33, 4, 10, "uniform", "plain"),
    (40, 4, 12, "uniform", "large")])
def test_beta_select_matches_oracle(N, R, G, kind, sweep):
    from paper_2605_24408_amd import pdit as P
    say(f"beta_select N={N} R={R} G={G} kind={kind} sweep={sweep}")
    rng = np.random.default_rng(N + G)
    if kind == "grid":
        inst = W.config_n12(R=R, T=1)
        D, F = inst.D, inst.F
    else:
        D, F = W.random_instance(rng, N, 0, 40, zero_diag=(kind != "diag"))
    perms = W.random_perms(rng, R, N)
    s = W.energy_scale(D, F)
    grid = np.geomspace(0.02 / s, 200.0 / s, G).astype(np.float32)
    trials, seed, L = 30, 21, 10
    ref = oracle.beta_select(D, F, perms, grid, trials, seed, L)
    with P.Pdit(sweep=sweep) as ctx:
        got = gpu_select(ctx, D, F, perms, grid, trials, seed, L)
        plan = ctx.last_plan()
    assert plan["sweep"] == (sweep if sweep in ("plain", "large") else "fast")
    assert np.array_equal(got["perm_after"], perms)  # the caller's permutations are untouched
    bad = np.nonzero(got["E"] != ref.E_trial.reshape(-1))[0]
    if bad.size:
        tied = tied_rows(D, F, perms, grid, trials, seed)
        assert set(bad.tolist()) <= tied, f"trial replicas {bad} differ without a counted tie"
        return
    assert np.array_equal(got["E_sum"], ref.E_sum)
    assert got["range"] == (ref.lo, ref.hi)
    assert np.array_equal(got["ladder"], ref.ladder)
    assert got["counters"][:, 0].sum() == G * R * N * trials


def test_beta_select_full_size_sampled():
    """The N=64 benchmark instance: 24 grid values x 64 trial replicas x 400
    sweeps in one launch; sampled trial replicas rerun on the oracle, the
    sums and the rule recomputed from every replica's energy."""
    from paper_2605_24408_amd import pdit as P
    inst = W.config_n64(R=64)
    s = W.energy_scale(inst.D, inst.F)
    grid = np.geomspace(0.01 / s, 100.0 / s, 24).astype(np.float32)
    G, R, trials, seed = 24, 64, 400, 3
    with P.Pdit() as ctx:
        got = gpu_select(ctx, inst.D, inst.F, inst.perms, grid, trials, seed, 10)
    E = got["E"].reshape(G, R)
    assert np.array_equal(got["E_sum"], E.sum(axis=1))
    lo, hi, ladder = oracle.beta_rule(got["E_sum"], grid, 10)
    assert got["range"] == (lo, hi) and np.array_equal(got["ladder"], ladder)
    assert lo < hi
    for g, k in ((0, 5), (G // 2, 17), (hi, 63)):
        ref = oracle.run(inst.D, inst.F, inst.perms[k:k + 1], np.full(trials, grid[g], np.float32),
                         seed, rep_ids=[g * R + k])
        if ref.counters[0][2] == 0:
            assert E[g, k] == ref.E[0], (g, k)


def test_selected_ladder_drives_parallel_tempering():
    """The chosen ladder is a valid pdit_pt ladder: one selection, then a
    fused parallel-tempering run on it equals the oracle's run_pt."""
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(31)
    N, L = 24, 6
    D, F = W.random_instance(rng, N, 0, 30)
    s = W.energy_scale(D, F)
    grid = np.geomspace(0.02 / s, 200.0 / s, 14).astype(np.float32)
    perms = W.random_perms(rng, 2 * L, N)
    with P.Pdit() as ctx:
        sel = gpu_select(ctx, D, F, perms[:4], grid, 40, 5, L)
        ladder = sel["ladder"]
        assert np.all(np.diff(ladder) > 0)
        p = dev(perms, torch.int32)
        slot = dev(np.tile(np.arange(L), 2), torch.int32)
        since = dev(np.zeros(2), torch.int32)
        ctx.run_pt(dev(D, torch.int32), dev(F, torch.int32), p, dev(ladder, torch.float32), slot,
                   since, 10, 4, 3, 9, "fused")
        got_perm = p.cpu().numpy()
    ref = oracle.run_pt(D, F, perms, ladder, 10, 4, 3, 9)
    if ref.counters[:, 2].sum() == 0:
        assert np.array_equal(got_perm, ref.perm)
        assert np.array_equal(slot.cpu().numpy(), ref.slot)


def test_beta_select_error_paths():
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(2)
    N = 10
    D, F = W.random_instance(rng, N, 0, 9)
    perms = W.random_perms(rng, 3, N)
    with P.Pdit() as ctx:
        for grid in ([0.1, 0.1, 0.2], [0.3, 0.2], [0.0, 0.1], [0.1, float("nan")], [-0.1, 0.2]):
            with pytest.raises(P.PditError) as e:
                gpu_select(ctx, D, F, perms, np.array(grid, np.float32), 5, 1, 4)
            assert e.value.status == "PDIT_EBETA", grid
        with pytest.raises(P.PditError) as e:
            gpu_select(ctx, D, F, perms, np.array([0.1, 0.2], np.float32), 5, 1, 1)
        assert e.value.status == "PDIT_EINVAL"
        bad = perms.copy()
        bad[1, 0] = bad[1, 1]
        with pytest.raises(P.PditError) as e:
            gpu_select(ctx, D, F, bad, np.array([0.1, 0.2], np.float32), 5, 1, 4)
        assert e.value.status == "PDIT_EBADPERM"
    # sums beyond 2^59: large values and many trial replicas
    D2 = W.sym_uniform(rng, 64, 0, 2_000_000).astype(np.int64)
    F2 = W.sym_uniform(rng, 64, 0, 2_000_000).astype(np.int64)
    with P.Pdit(sweep="plain") as ctx:
        with pytest.raises(P.PditError) as e:
            gpu_select(ctx, D2, F2, W.random_perms(rng, 4096, 64), np.array([1e-9, 2e-9], np.float32),
                       1, 1, 3)
        assert e.value.status == "PDIT_EOVERFLOW"
