"""Beta-range selection on the GPU (pdit_beta_select) against the oracle's
beta_select: every trial replica's ending energy, the summed energies, the
chosen range and the ladder, on each sweep kernel; the ladder feeding a
parallel-tempering run; error paths.

The selection's launch does not record draws.  Each grid value's trials are
therefore run again as a recorded single-instance run whose rows g R + k
carry the trials' Philox replica indices; those rows must end where the
selection's trials ended, and they are replayed draw by draw on the oracle
(``parity.py``).  The rule must then equal the oracle's rule on the GPU's
sums, and the whole selection the oracle's when no draw was adopted at a
tie."""
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


def gpu_select(ctx, D, F, perms, grid, trials, seed, L, level=40):
    Dd, Fd, pd = dev(D, torch.int32), dev(F, torch.int32), dev(perms, torch.int32)
    E_sum, ladder, rng = ctx.beta_select(Dd, Fd, pd, dev(grid, torch.float32), trials, seed, L,
                                         level)
    out = {"E_sum": E_sum.cpu().numpy(), "ladder": ladder.cpu().numpy(),
           "range": tuple(int(x) for x in rng.cpu().numpy()), "E": ctx.energy().cpu().numpy(),
           "counters": ctx.replica_counters().cpu().numpy(), "perm_after": pd.cpu().numpy()}
    return out


def replay_trials(P, sweep, D, F, perms, grid, trials, seed, E_trial, g, ks, what):
    """Trial replicas (g, k) for k in ks: a recorded single-instance run of
    (g + 1) R rows (row g R + k starts from perms[k] and draws as replica
    g R + k) at beta grid[g]; rows g R + k must end at the selection's
    energies and are replayed on the oracle.  Returns the draws adopted at
    ties."""
    R, N = perms.shape
    tiled = np.tile(perms, (g + 1, 1))
    beta = np.full(trials, grid[g], np.float32)
    with P.Pdit(sweep=sweep) as ctx:
        p = dev(tiled, torch.int32)
        ch = torch.full((tiled.shape[0], trials, N), -1, dtype=torch.int32, device=DEV)
        tr = torch.zeros((tiled.shape[0], trials), dtype=torch.int64, device=DEV)
        ctx.set_recording(ch, tr)
        ctx.run_sweeps(dev(D, torch.int32), dev(F, torch.int32), p, dev(beta, torch.float32), seed)
        Eb, pb = ctx.best()
        rows = [g * R + k for k in ks]
        got = {"perm": p.cpu().numpy(), "E": ctx.energy().cpu().numpy(),
               "E_best": Eb.cpu().numpy(), "perm_best": pb.cpu().numpy(),
               "counters": ctx.replica_counters().cpu().numpy(),
               "choices": ch.cpu().numpy(), "trace": tr.cpu().numpy()}
    for k in ks:
        assert got["E"][g * R + k] == E_trial[g * R + k], (g, k)
    parts = replay(got, D, F, perms[list(ks)], beta, seed, rows=rows, what=f"{what} grid {g}")
    return sum(int(x.excused[0]) for x in parts)


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
    for level in (40, 60):
        ref = oracle.beta_select(D, F, perms, grid, trials, seed, L, level_pct=level)
        with P.Pdit(sweep=sweep) as ctx:
            got = gpu_select(ctx, D, F, perms, grid, trials, seed, L, level)
            plan = ctx.last_plan()
        assert plan["sweep"] == (sweep if sweep in ("plain", "large") else "fast")
        assert np.array_equal(got["perm_after"], perms)  # the caller's permutations are untouched
        assert got["counters"][:, 0].sum() == G * R * N * trials
        E = got["E"].reshape(G, R)
        assert np.array_equal(got["E_sum"], E.sum(axis=1))
        lo, hi, ladder = oracle.beta_rule(got["E_sum"], grid, L, level)
        assert got["range"] == (lo, hi) and np.array_equal(got["ladder"], ladder)
    adopted = sum(replay_trials(P, sweep, D, F, perms, grid, trials, seed, got["E"], g, range(R),
                                f"beta_select N={N}") for g in range(G))
    if adopted == 0:
        assert np.array_equal(got["E"], ref.E_trial.reshape(-1))
        assert np.array_equal(got["E_sum"], ref.E_sum)
        assert got["range"] == (ref.lo, ref.hi)
        assert np.array_equal(got["ladder"], ref.ladder)


def test_beta_select_full_size_sampled():
    """The N=64 benchmark instance: 24 grid values x 64 trial replicas x 400
    sweeps in one launch; sampled trial replicas replayed on the oracle
    (recorded reruns), the sums and the rule recomputed from every
    replica's energy."""
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
        replay_trials(P, "auto", inst.D, inst.F, inst.perms, grid, trials, seed, got["E"], g, [k],
                      "beta_select n64")


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
    from test_gpu_pt import pt_chunked
    chunked, _ = pt_chunked(P, D, F, perms, ladder, 10, 4, 3, 9, 2, schedule="fused",
                            what="pt on the selected ladder")
    assert np.array_equal(got_perm, chunked["perm"])
    assert np.array_equal(slot.cpu().numpy(), chunked["slot"])


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
