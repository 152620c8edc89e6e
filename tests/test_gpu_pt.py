"""Parallel tempering on the GPU (pdit_run_pt) against the oracle's
run_pt: every sweep kernel, resume across calls, forced top-bottom trades,
exchange-only periods and the error paths.  Tempering launches do not
record their draws, so parity is checked chunk by chunk (``parity.py``):
after every few periods each set (its replicas' states, energies, best
states and counters, its slots and pass counter) must equal an oracle run
of the same periods from the same state, unless the oracle counted a tie in
that set during those periods; the oracle is then re-synced to the GPU's
state."""
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


def gpu_pt(ctx, D, F, perms, ladder, periods, per_sweeps, timeout, seed, slot=None, since=None,
           schedule="auto", dynamics="sequential"):
    L = len(ladder)
    R = perms.shape[0]
    p = dev(perms, torch.int32)
    sl = dev(np.tile(np.arange(L), R // L) if slot is None else slot, torch.int32)
    st = dev(np.zeros(R // L) if since is None else since, torch.int32)
    ctx.run_pt(dev(D, torch.int32), dev(F, torch.int32), p, dev(ladder, torch.float32), sl, st,
               periods, per_sweeps, timeout, seed, schedule, dynamics)
    E_best, perm_best = ctx.best()
    return {"perm": p.cpu().numpy(), "E": ctx.energy().cpu().numpy(),
            "E_best": E_best.cpu().numpy(), "perm_best": perm_best.cpu().numpy(),
            "counters": ctx.replica_counters().cpu().numpy(), "slot": sl.cpu().numpy(),
            "since_top": st.cpu().numpy()}


def set_differs(got, ref, g, L):
    rows = range(g * L, (g + 1) * L)
    same = all(np.array_equal(got["perm"][k], ref.perm[k]) and got["E"][k] == ref.E[k]
               and got["E_best"][k] == ref.E_best[k]
               and np.array_equal(got["perm_best"][k], ref.perm_best[k])
               and np.array_equal(got["counters"][k][:2], ref.counters[k][:2]) for k in rows)
    same = same and np.array_equal(got["slot"][g * L:(g + 1) * L], ref.slot[g * L:(g + 1) * L])
    return not (same and got["since_top"][g] == ref.since_top[g])


def pt_chunked(P, D, F, perms, ladder, periods, per, timeout, seed, chunk, sweep="auto",
               schedule="auto", dynamics="sequential", what="pt"):
    """The GPU run in calls of ``chunk`` periods, each compared set by set
    with the oracle's run of the same periods from the GPU's previous state
    (a set may differ only with an oracle tie in it during those periods).
    Returns the final GPU state and the plan."""
    L = len(ladder)
    R = perms.shape[0]
    method = "cupim" if dynamics == "cupim" else "sequential"
    state = {"perm": perms, "slot": np.tile(np.arange(L), R // L), "since_top": np.zeros(R // L),
             "E_best": None, "perm_best": None}
    resync = 0
    with P.Pdit(sweep=sweep) as ctx:
        p = dev(perms, torch.int32)
        sl = dev(state["slot"], torch.int32)
        st = dev(state["since_top"], torch.int32)
        Dd, Fd, ld = dev(D, torch.int32), dev(F, torch.int32), dev(ladder, torch.float32)
        done = 0
        while done < periods:
            k = min(chunk, periods - done)
            ctx.run_pt(Dd, Fd, p, ld, sl, st, k, per, timeout, seed, schedule, dynamics)
            E_best, perm_best = ctx.best()
            got = {"perm": p.cpu().numpy(), "E": ctx.energy().cpu().numpy(),
                   "E_best": E_best.cpu().numpy(), "perm_best": perm_best.cpu().numpy(),
                   "counters": ctx.replica_counters().cpu().numpy(), "slot": sl.cpu().numpy(),
                   "since_top": st.cpu().numpy()}
            ref = oracle.run_pt(D, F, state["perm"], ladder, k, per, timeout, seed,
                                sweep_offset=done * per, slot=state["slot"],
                                since_top=state["since_top"], E_best=state["E_best"],
                                perm_best=state["perm_best"], method=method)
            for g in range(R // L):
                if set_differs(got, ref, g, L):
                    assert ref.counters[g * L:(g + 1) * L, 2].sum() > 0, (
                        f"{what}: periods {done}..{done + k}, set {g} differs from the oracle "
                        f"with no oracle tie in it")
                    resync += 1
            state = got
            done += k
        plan = ctx.last_plan()
    say(f"{what}: {periods} periods in chunks of {chunk}, {resync} set re-syncs at oracle ties")
    assert resync <= max(1, (R // L) * periods // (4 * chunk))
    return state, plan


TABLE_CASES = [(12, 4, 3, "fast", "grid"), (16, 4, 2, "fast", "uniform"),
               (40, 5, 2, "fast", "uniform"), (128, 4, 1, "fast", "uniform"),
               (64, 10, 2, "fast", "uniform"), (64, 6, 2, "fast", "diag"), (100, 3, 2, "fast", "diag")]


@pytest.mark.parametrize("N,L,sets,sweep,kind,schedule",
                         [c + (s,) for c in TABLE_CASES for s in ("periodic", "fused")]
                         + [(140, 4, 2, "fast", "uniform", "auto"),
                            (33, 5, 2, "plain", "uniform", "auto"),
                            (33, 5, 2, "large", "uniform", "auto"),
                            (200, 3, 1, "large", "diag", "auto")])
def test_pt_matches_oracle(N, L, sets, sweep, kind, schedule):
    from paper_2605_24408_amd import pdit as P
    say(f"pt N={N} L={L} sets={sets} sweep={sweep} kind={kind} schedule={schedule}")
    rng = np.random.default_rng(N * 3 + L)
    if kind == "grid":
        inst = W.config_n12(R=L * sets, T=1)
        D, F = inst.D, inst.F
    else:
        D, F = W.random_instance(rng, N, 0, 40, zero_diag=(kind != "diag"))
    perms = W.random_perms(rng, L * sets, N)
    s = W.energy_scale(D, F)
    ladder = W.beta_geometric(0.5 / s, 60.0 / s, L)
    periods, per, timeout = 12, 4, 3
    got, plan = pt_chunked(P, D, F, perms, ladder, periods, per, timeout, 17, 3, sweep=sweep,
                           schedule=schedule, what=f"pt N={N} {sweep} {schedule}")
    assert plan["sweep"] == sweep
    assert got["counters"][:, 1].sum() > 0


@pytest.mark.parametrize("schedule", ["periodic", "fused"])
def test_pt_resume_equals_single_call(schedule):
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(5)
    N, L = 48, 6
    D, F = W.random_instance(rng, N, 0, 30)
    perms = W.random_perms(rng, 2 * L, N)
    s = W.energy_scale(D, F)
    ladder = W.beta_geometric(1.0 / s, 40.0 / s, L)
    with P.Pdit() as ctx:
        one = gpu_pt(ctx, D, F, perms, ladder, 10, 4, 2, 3, schedule=schedule)
    with P.Pdit() as ctx:
        a = gpu_pt(ctx, D, F, perms, ladder, 6, 4, 2, 3, schedule=schedule)
        b = gpu_pt(ctx, D, F, a["perm"], ladder, 4, 4, 2, 3, slot=a["slot"], since=a["since_top"],
                   schedule=schedule)
    for f in ("perm", "E", "E_best", "perm_best", "slot", "since_top"):
        assert np.array_equal(one[f], b[f]), f


@pytest.mark.parametrize("N,L,sets,periods,per_sweeps,timeout", [
    (64, 10, 102, 40, 4, 5), (128, 4, 70, 6, 3, 2), (20, 64, 40, 30, 2, 7), (32, 1, 300, 5, 3, 2)])
def test_pt_fused_equals_periodic(N, L, sets, periods, per_sweeps, timeout):
    """Full-size ladders: the fused launch (whole sets per cooperative
    launch; 280 replicas of N = 128 need two launches) against one launch per
    period, every output equal."""
    from paper_2605_24408_amd import pdit as P
    say(f"pt fused vs periodic N={N} L={L} sets={sets}")
    rng = np.random.default_rng(N + L)
    D, F = W.random_instance(rng, N, 0, 99)
    perms = W.random_perms(rng, L * sets, N)
    s = W.energy_scale(D, F)
    ladder = W.beta_geometric(0.3 / s, 30.0 / s, L)
    with P.Pdit() as ctx:
        a = gpu_pt(ctx, D, F, perms, ladder, periods, per_sweeps, timeout, 11, schedule="periodic")
        ca = ctx.counters()
    with P.Pdit() as ctx:
        b = gpu_pt(ctx, D, F, perms, ladder, periods, per_sweeps, timeout, 11, schedule="fused")
        cb = ctx.counters()
    for f in ("perm", "E", "E_best", "perm_best", "counters", "slot", "since_top"):
        assert np.array_equal(a[f], b[f]), f
    assert ca == cb and ca["accepted"] > 0
    for g in range(sets):
        assert sorted(b["slot"][g * L:(g + 1) * L]) == list(range(L))


def test_pt_exchange_only_periods():
    """period_sweeps = 0: the passes act on the recomputed energies alone."""
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(9)
    N, L = 20, 8
    D, F = W.random_instance(rng, N, 0, 9)
    perms = W.random_perms(rng, 3 * L, N)
    ladder = np.linspace(0.1, 0.8, L).astype(np.float32)
    ref = oracle.run_pt(D, F, perms, ladder, 7, 0, 2, 1)
    with P.Pdit() as ctx:
        got = gpu_pt(ctx, D, F, perms, ladder, 7, 0, 2, 1)
    assert np.array_equal(got["slot"], ref.slot) and np.array_equal(got["since_top"], ref.since_top)
    assert np.array_equal(got["perm"], perms)


def test_pt_error_paths():
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(2)
    N, L = 16, 4
    D, F = W.random_instance(rng, N, 0, 9)
    perms = W.random_perms(rng, 2 * L, N)
    ladder = np.linspace(0.1, 1.0, L).astype(np.float32)
    with P.Pdit() as ctx:
        for slot, why in ((np.array([0, 1, 2, 2, 0, 1, 2, 3]), "repeated rung"),
                          (np.array([0, 1, 2, 4, 0, 1, 2, 3]), "rung out of range")):
            with pytest.raises(P.PditError) as e:
                gpu_pt(ctx, D, F, perms, ladder, 1, 1, 5, 1, slot=slot)
            assert e.value.status == "PDIT_EINVAL", why
        with pytest.raises(P.PditError) as e:
            gpu_pt(ctx, D, F, perms[:7], ladder, 1, 1, 5, 1, slot=np.arange(7) % L)
        assert e.value.status == "PDIT_EINVAL"
        with pytest.raises(P.PditError) as e:
            gpu_pt(ctx, D, F, perms, np.array([0.1, -1.0, 0.2, 0.3], np.float32), 1, 1, 5, 1)
        assert e.value.status == "PDIT_EBETA"
    # the fused schedule needs the table kernel
    with P.Pdit(sweep="plain") as ctx:
        with pytest.raises(P.PditError) as e:
            gpu_pt(ctx, D, F, perms, ladder, 1, 1, 5, 1, schedule="fused")
        assert e.value.status == "PDIT_EINVAL"
    rng = np.random.default_rng(3)
    D2, F2 = W.random_instance(rng, 140, 0, 9)
    with P.Pdit() as ctx:
        with pytest.raises(P.PditError) as e:
            gpu_pt(ctx, D2, F2, W.random_perms(rng, 4, 140), ladder, 1, 1, 5, 1, schedule="fused")
        assert e.value.status == "PDIT_EINVAL"


@pytest.mark.parametrize("N,L,sets,kind", [(12, 4, 3, "grid"), (40, 5, 2, "uniform"),
                                           (64, 10, 2, "uniform"), (100, 3, 2, "diag"),
                                           (128, 4, 1, "uniform")])
def test_pt_cupim_matches_oracle(N, L, sets, kind):
    """Parallel tempering with concurrent updates (Methods, "GPU-CUPIM
    Algorithm") against the oracle's run_pt(method="cupim")."""
    from paper_2605_24408_amd import pdit as P
    say(f"pt cupim N={N} L={L} sets={sets} kind={kind}")
    rng = np.random.default_rng(N * 5 + L)
    if kind == "grid":
        inst = W.config_n12(R=L * sets, T=1)
        D, F = inst.D, inst.F
    else:
        D, F = W.random_instance(rng, N, 0, 99, zero_diag=(kind != "diag"))
    perms = W.random_perms(rng, L * sets, N)
    s = W.energy_scale(D, F)
    ladder = W.beta_geometric(0.5 / s, 60.0 / s, L)
    got, _ = pt_chunked(P, D, F, perms, ladder, 10, 4, 3, 23, 2, dynamics="cupim",
                        what=f"pt cupim N={N}")
    assert got["counters"][:, 1].sum() > 0


def test_pt_cupim_resume_and_errors():
    from paper_2605_24408_amd import pdit as P
    rng = np.random.default_rng(8)
    N, L = 30, 5
    D, F = W.random_instance(rng, N, 0, 50)
    perms = W.random_perms(rng, 2 * L, N)
    s = W.energy_scale(D, F)
    ladder = W.beta_geometric(0.5 / s, 30.0 / s, L)
    with P.Pdit() as ctx:
        one = gpu_pt(ctx, D, F, perms, ladder, 8, 3, 2, 5, dynamics="cupim")
    with P.Pdit() as ctx:
        a = gpu_pt(ctx, D, F, perms, ladder, 5, 3, 2, 5, dynamics="cupim")
        b = gpu_pt(ctx, D, F, a["perm"], ladder, 3, 3, 2, 5, slot=a["slot"], since=a["since_top"],
                   dynamics="cupim")
    for f in ("perm", "E", "E_best", "perm_best", "slot", "since_top"):
        assert np.array_equal(one[f], b[f]), f
    with P.Pdit() as ctx:
        with pytest.raises(P.PditError) as e:
            gpu_pt(ctx, D, F, perms, ladder, 1, 1, 2, 1, schedule="fused", dynamics="cupim")
        assert e.value.status == "PDIT_EINVAL"
        D2, F2 = W.random_instance(rng, N, 0, 300)
        with pytest.raises(P.PditError) as e:
            gpu_pt(ctx, D2, F2, perms, ladder, 1, 1, 2, 1, dynamics="cupim")
        assert e.value.status == "PDIT_EOVERFLOW"
