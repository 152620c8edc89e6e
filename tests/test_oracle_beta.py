"""Pins of the oracle's beta-range selection (Results, "Implementation";
Methods, "CPU-PIM Algorithm"): the range rule on hand-worked sums, the
geometric ladder, the trials as a composition of the pinned sweep, the
beta -> 0 trial against the closed-form mean energy of a uniformly random
permutation, and the large-beta trial ending in 2-opt local minima."""
import itertools
import json
import os

import numpy as np
import pytest

import oracle
from paper_2605_24408_amd import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "beta_rule.json")


def test_rule_hand_cases():
    cases = json.load(open(GOLDEN))["cases"]
    for c in cases:
        G = len(c["sums"])
        grid = np.geomspace(0.01, 10.0, G).astype(np.float32) if G > 1 else np.array([0.5], np.float32)
        lo, hi, ladder = oracle.beta_rule(c["sums"], grid, 6, c["level_pct"])
        assert (lo, hi) == (c["lo"], c["hi"]), c["why"]
        assert ladder[0] == grid[lo] and ladder[-1] == grid[hi]


@pytest.mark.parametrize("L", [2, 3, 10, 64])
def test_ladder_is_geometric(L):
    grid = np.geomspace(1e-4, 3.0, 30).astype(np.float32)
    sums = np.array([1000 - 30 * g + (g > 20) * 40 * (g - 20) for g in range(30)], np.int64)
    lo, hi, ladder = oracle.beta_rule(sums, grid, L)
    assert lo < hi
    r = (float(grid[hi]) / float(grid[lo])) ** (1.0 / (L - 1))
    ratios = ladder[1:].astype(np.float64) / ladder[:-1].astype(np.float64)
    assert np.all(np.abs(ratios / r - 1.0) < 1e-6)
    assert ladder[0] == grid[lo] and ladder[-1] == grid[hi]


def test_rule_level_is_monotone():
    """A higher level (further above the minimum) never picks a later low end;
    levels 40 and 60 (the two readings of the paper's wording) pick
    different low ends on a steadily falling curve."""
    rng = np.random.default_rng(3)
    grid = np.geomspace(0.01, 10.0, 20).astype(np.float32)
    for _ in range(200):
        sums = np.sort(rng.integers(-10**9, 10**9, size=20))[::-1].copy()
        los = [oracle.beta_rule(sums, grid, 4, lv)[0] for lv in (0, 20, 40, 60, 80, 100)]
        assert los == sorted(los, reverse=True)
    sums = np.arange(20, 0, -1) * 1000
    assert oracle.beta_rule(sums, grid, 4, 40)[0] > oracle.beta_rule(sums, grid, 4, 60)[0]


def test_rule_rejects_bad_input():
    grid = np.array([0.1, 0.2], np.float32)
    with pytest.raises(RuntimeError):
        oracle.beta_rule([1, 2], grid, 3, 101)   # level beyond the range
    with pytest.raises(RuntimeError):
        oracle.beta_rule([1, 2], grid, 1)       # a ladder needs two rungs
    with pytest.raises(RuntimeError):
        oracle.beta_rule([1 << 60, 2], grid, 3)  # sums beyond 2^59
    rng = np.random.default_rng(0)
    D, F = W.random_instance(rng, 6, 0, 5)
    perms = W.random_perms(rng, 2, 6)
    for bad in ([0.0, 0.1], [0.2, 0.1], [0.1, 0.1], [0.1, np.inf]):
        with pytest.raises(RuntimeError):
            oracle.beta_select(D, F, perms, np.array(bad, np.float32), 3, 1, 3)


def test_trials_compose_the_pinned_sweep():
    """E_sum[g] is the sum of plain runs at grid[g] with replica ids g R + k."""
    rng = np.random.default_rng(4)
    N, R = 9, 5
    D, F = W.random_instance(rng, N, 0, 9)
    perms = W.random_perms(rng, R, N)
    grid = np.geomspace(0.01, 2.0, 6).astype(np.float32)
    sel = oracle.beta_select(D, F, perms, grid, 20, 7, 4)
    for g, b in enumerate(grid):
        ref = oracle.run(D, F, perms, np.full(20, b, np.float32), 7,
                         rep_ids=[g * R + k for k in range(R)])
        assert np.array_equal(sel.E_trial[g], ref.E)
        assert sel.E_sum[g] == ref.E.sum()
    lo, hi, ladder = oracle.beta_rule(sel.E_sum, grid, 4)
    assert (lo, hi) == (sel.lo, sel.hi) and np.array_equal(ladder, sel.ladder)


def test_hot_trial_mean_is_the_uniform_permutation_mean():
    """At beta -> 0 every candidate is equally likely, the chain is a lazy
    random-transposition walk and its ending permutation is uniform: the
    mean ending energy is the closed form
    (sum_{i!=j} D_ij)(sum_{a!=b} F_ab) / (N (N-1)) + (sum_i D_ii)(sum_a F_aa) / N."""
    rng = np.random.default_rng(8)
    N, R = 7, 3000
    D, F = W.random_instance(rng, N, 0, 9, zero_diag=False)
    perms = np.tile(np.arange(N, dtype=np.int32), (R, 1))  # every trial from the identity
    Di, Fi = D.astype(np.int64), F.astype(np.int64)
    off = lambda M: M.sum() - np.trace(M)
    mean = off(Di) * off(Fi) / (N * (N - 1)) + np.trace(Di) * np.trace(Fi) / N
    # spread of E over all N! permutations (exact, by enumeration)
    Es = np.array([(Di * Fi[np.ix_(p, p)]).sum() for p in itertools.permutations(range(N))])
    assert abs(Es.mean() - mean) < 1e-9 * abs(mean)
    sel = oracle.beta_select(D, F, perms, np.array([1e-9], np.float32), 40, 3, 2)
    got = sel.E_trial[0].mean()
    assert abs(got - mean) < 5 * Es.std() / np.sqrt(R)
    # a cold trial from the identity ends among the lowest 1% of all N!
    # energies, at or above the exhaustive minimum
    cold = oracle.beta_select(D, F, perms[:200], np.array([5.0], np.float32), 40, 3, 2)
    assert cold.E_trial[0].min() >= Es.min()
    assert np.mean(Es <= cold.E_trial[0].max()) < 0.01


def test_frozen_trial_ends_in_two_opt_minima():
    """At a very large beta only energy-lowering (or equal) exchanges are
    taken, so after enough sweeps no exchange of two locations lowers
    Eq. 1 (checked by recomputing Eq. 1 for every exchange)."""
    rng = np.random.default_rng(12)
    N, R = 10, 6
    D, F = W.random_instance(rng, N, 0, 20)
    perms = W.random_perms(rng, R, N)
    res = oracle.run(D, F, perms, np.full(200, 1e3, np.float32), 5,
                     rep_ids=list(range(R)))
    Di, Fi = D.astype(np.int64), F.astype(np.int64)
    energy = lambda p: int((Di * Fi[np.ix_(p, p)]).sum())
    for p, e in zip(res.perm, res.E):
        assert energy(p) == e
        for i, j in itertools.combinations(range(N), 2):
            q = p.copy()
            q[i], q[j] = q[j], q[i]
            assert energy(q) >= e
    sel = oracle.beta_select(D, F, perms, np.array([1e3], np.float32), 200, 5, 2)
    assert np.array_equal(sel.E_trial[0], res.E)
