"""Pins of the oracle's parallel tempering (Results, "Implementation";
Methods, "CPU-PIM Algorithm"): the exchange pass on hand-worked cases, and
the driver as a composition of pinned parts."""
import json
import os

import numpy as np

import oracle
from paper_2605_24408_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "pt_exchange.json")


def test_exchange_hand_cases():
    cases = json.load(open(GOLDEN))["cases"]
    assert len(cases) >= 6
    for c in cases:
        sl, st, top = oracle.pt_exchange(c["energy"], c["slot_of"], c["since_top"], c["timeout"])
        assert list(sl) == c["expect_slot_of"], c["name"]
        assert st == c["expect_since_top"], c["name"]
        assert top == c["expect_top_changed"], c["name"]


def test_exchange_keeps_slots_a_permutation():
    rng = np.random.default_rng(4)
    for L in (1, 2, 3, 10):
        sl, st = np.arange(L, dtype=np.int32), 0
        for _ in range(300):
            E = rng.integers(-5, 5, L)
            sl, st, _ = oracle.pt_exchange(E, sl, st, 7)
            assert sorted(sl) == list(range(L)) and 0 <= st < 7


def test_single_slot_ladder_is_a_constant_beta_run():
    """L = 1: no exchange can move anything; the run equals po_run at the
    slot's beta over n_periods * period_sweeps sweeps."""
    rng = np.random.default_rng(1)
    D, F = W.random_instance(rng, 9, 0, 9)
    perms = W.random_perms(rng, 3, 9)
    s = W.energy_scale(D, F)
    b = np.float32(3.0 / s)
    pt = oracle.run_pt(D, F, perms, [b], n_periods=6, period_sweeps=4, timeout=2, seed=5)
    ref = oracle.run(D, F, perms, np.full(24, b, np.float32), 5)
    assert np.array_equal(pt.perm, ref.perm) and np.array_equal(pt.E, ref.E)
    assert np.array_equal(pt.E_best, ref.E_best) and np.array_equal(pt.counters, ref.counters)


def test_driver_composes_sweeps_and_exchanges():
    """One period by hand: every replica runs period_sweeps sweeps at its
    slot's beta (its own random stream, the global sweep index), then each
    set runs one exchange pass on the resulting energies."""
    rng = np.random.default_rng(2)
    N, L, sets, per = 8, 4, 2, 3
    D, F = W.random_instance(rng, N, 0, 9)
    perms = W.random_perms(rng, L * sets, N)
    s = W.energy_scale(D, F)
    ladder = W.beta_geometric(0.2 / s, 20.0 / s, L)
    slot = np.array([2, 0, 3, 1, 0, 1, 2, 3], np.int32)
    since = np.array([5, 0], np.int32)
    pt = oracle.run_pt(D, F, perms, ladder, 1, per, 100, 9, sweep_offset=40, slot=slot,
                       since_top=since)
    perm = perms.copy()
    E = np.zeros(L * sets, np.int64)
    for k in range(L * sets):
        r = oracle.run(D, F, perm[k:k + 1], np.full(per, ladder[slot[k]], np.float32), 9,
                       sweep_offset=40, rep_ids=[k])
        perm[k] = r.perm[0]
        E[k] = r.E[0]
    assert np.array_equal(pt.perm, perm) and np.array_equal(pt.E, E)
    for g in range(sets):
        sl, st, _ = oracle.pt_exchange(E[g * L:(g + 1) * L], slot[g * L:(g + 1) * L], since[g], 100)
        assert np.array_equal(pt.slot[g * L:(g + 1) * L], sl) and pt.since_top[g] == st


def test_resume_equals_single_run():
    rng = np.random.default_rng(3)
    N, L = 10, 5
    D, F = W.random_instance(rng, N, 0, 20)
    perms = W.random_perms(rng, 2 * L, N)
    s = W.energy_scale(D, F)
    ladder = W.beta_geometric(0.3 / s, 30.0 / s, L)
    full = oracle.run_pt(D, F, perms, ladder, 9, 4, 3, 11)
    a = oracle.run_pt(D, F, perms, ladder, 5, 4, 3, 11)
    b = oracle.run_pt(D, F, a.perm, ladder, 4, 4, 3, 11, sweep_offset=20, slot=a.slot,
                      since_top=a.since_top, E_best=a.E_best, perm_best=a.perm_best)
    for f in ("perm", "E", "E_best", "perm_best", "slot", "since_top"):
        assert np.array_equal(getattr(full, f), getattr(b, f)), f
    assert np.array_equal(full.counters, a.counters + b.counters)


def test_invariants_and_energies():
    rng = np.random.default_rng(6)
    N, L = 11, 6
    D, F = W.random_instance(rng, N, 0, 30, zero_diag=False)
    perms = W.random_perms(rng, 2 * L, N)
    s = W.energy_scale(D, F)
    pt = oracle.run_pt(D, F, perms, W.beta_geometric(0.5 / s, 50.0 / s, L), 12, 4, 5, 3)
    for k in range(2 * L):
        assert sorted(pt.perm[k]) == list(range(N))
        assert pt.E[k] == oracle.energy(D, F, pt.perm[k])
        assert pt.E_best[k] == oracle.energy(D, F, pt.perm_best[k]) <= pt.E[k]
    for g in range(2):
        assert sorted(pt.slot[g * L:(g + 1) * L]) == list(range(L))


def test_reaches_the_brute_force_minimum():
    """Small instance: one set of 6 replicas finds the exhaustive optimum."""
    rng = np.random.default_rng(8)
    N = 7
    D, F = W.random_instance(rng, N, 0, 9)
    best, _ = oracle.brute_min(D, F)
    s = W.energy_scale(D, F)
    pt = oracle.run_pt(D, F, W.random_perms(rng, 6, N), W.beta_geometric(0.5 / s, 40.0 / s, 6),
                       60, 4, 100, 1)
    assert pt.E_best.min() == best


def test_cupim_dynamics_single_rung_is_a_cupim_run():
    """Parallel tempering with the GPU-CUPIM iteration (Methods, "GPU-CUPIM
    Algorithm"): with L = 1 the run equals run_cupim at the rung's beta over
    n_periods * period_sweeps iterations."""
    rng = np.random.default_rng(11)
    D, F = W.random_instance(rng, 10, 0, 9)
    perms = W.random_perms(rng, 3, 10)
    s = W.energy_scale(D, F)
    b = np.float32(1.5 / s)
    pt = oracle.run_pt(D, F, perms, [b], 5, 4, 2, 7, method="cupim")
    ref = oracle.run_cupim(D, F, perms, np.full(20, b, np.float32), 7)
    assert np.array_equal(pt.perm, ref.perm) and np.array_equal(pt.E, ref.E)
    assert np.array_equal(pt.E_best, ref.E_best) and np.array_equal(pt.counters, ref.counters)


def test_cupim_dynamics_compose_with_exchanges():
    """One period by hand with the CUPIM iteration: every replica runs
    run_cupim at its rung's beta, then each set's exchange pass."""
    rng = np.random.default_rng(12)
    N, L, sets, per = 9, 3, 2, 4
    D, F = W.random_instance(rng, N, 0, 9)
    perms = W.random_perms(rng, L * sets, N)
    s = W.energy_scale(D, F)
    ladder = W.beta_geometric(0.2 / s, 20.0 / s, L)
    slot = np.array([1, 2, 0, 0, 2, 1], np.int32)
    since = np.array([0, 3], np.int32)
    pt = oracle.run_pt(D, F, perms, ladder, 1, per, 4, 3, sweep_offset=9, slot=slot,
                       since_top=since, method="cupim")
    perm = perms.copy()
    E = np.zeros(L * sets, np.int64)
    for k in range(L * sets):
        r = oracle.run_cupim(D, F, perm[k:k + 1], np.full(per, ladder[slot[k]], np.float32), 3,
                             sweep_offset=9, rep_ids=[k])
        perm[k] = r.perm[0]
        E[k] = r.E[0]
    assert np.array_equal(pt.perm, perm) and np.array_equal(pt.E, E)
    for g in range(sets):
        sl, st, _ = oracle.pt_exchange(E[g * L:(g + 1) * L], slot[g * L:(g + 1) * L], since[g], 4)
        assert np.array_equal(pt.slot[g * L:(g + 1) * L], sl) and pt.since_top[g] == st
