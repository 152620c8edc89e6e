"""Pins of the oracle's Gibbs choice (Eq. 5) and sweep dynamics: closed
forms, the one-step law against the exact softmax, and the long-run law
against the exact stationary vector of the one-sweep transition kernel."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats

from paper_2605_24408_amd import workloads as W

TWO24 = 1 << 24


def edge_u24(n, rng):
    base = [0, 1, 2, 15, 16, 17, TWO24 - 1, TWO24 - 2, TWO24 // 2, TWO24 // 3]
    return base + [int(v) for v in rng.integers(0, TWO24, size=n)]


@pytest.mark.parametrize("N", [2, 3, 5, 12, 64, 100, 512])
def test_beta_zero_is_uniform_index(orc, N):
    """beta = 0 makes every weight 1, so the choice is floor(u N)."""
    rng = np.random.default_rng(N)
    dE = rng.integers(-10**6, 10**6, size=N)
    for u in edge_u24(300, rng) + [(k * TWO24) // N for k in range(N)] + [(k * TWO24) // N - 1 for k in range(1, N)]:
        k, _ = orc.gibbs_choice(dE, 0.0, u)
        assert k == (u * N) >> 24


@pytest.mark.parametrize("N", [3, 17, 64])
def test_all_equal_deltas_any_beta(orc, N):
    """F = 0 (or a constant off-diagonal D) makes every energy change 0."""
    rng = np.random.default_rng(3)
    dE = np.zeros(N, dtype=np.int64)
    for beta in (0.0, 0.5, 1e3):
        for u in edge_u24(50, rng):
            assert orc.gibbs_choice(dE, beta, u)[0] == (u * N) >> 24


def test_frozen_unique_minimum(orc):
    rng = np.random.default_rng(4)
    for _ in range(50):
        N = int(rng.integers(2, 80))
        dE = rng.permutation(N * 3)[:N].astype(np.int64) - N
        for u in edge_u24(20, rng):
            assert orc.gibbs_choice(dE, 1e3, u)[0] == int(np.argmin(dE))


def test_frozen_tied_minimum_set(orc):
    """With a tied minimum set T and every other weight 0, the choice is
    T[floor(u |T|)]."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        N = int(rng.integers(3, 60))
        m = int(rng.integers(2, N + 1))
        T = np.sort(rng.choice(N, size=m, replace=False))
        dE = np.full(N, 1000, dtype=np.int64)
        dE[T] = -7
        for u in edge_u24(20, rng):
            assert orc.gibbs_choice(dE, 1.0, u)[0] == T[(u * m) >> 24]


def softmax64(dE, beta):
    x = -beta * (np.asarray(dE, dtype=np.float64) - np.min(dE))
    w = np.exp(x)
    return w / w.sum()


def chi2_pvalue(counts, probs):
    M = counts.sum()
    exp = probs * M
    keep = exp >= 5
    obs = np.append(counts[keep], counts[~keep].sum())
    ex = np.append(exp[keep], exp[~keep].sum())
    if ex[-1] == 0:
        obs, ex = obs[:-1], ex[:-1]
    ex = ex * obs.sum() / ex.sum()
    return stats.chisquare(obs, ex).pvalue


@pytest.mark.parametrize("N,scale", [(5, 0.5), (8, 1.0), (12, 2.0), (40, 1.0)])
def test_one_step_law_matches_softmax(orc, N, scale):
    """M independent draws of one p-dit update (distinct Philox counters)
    follow exp(-beta dE_k) / sum_j exp(-beta dE_j)."""
    rng = np.random.default_rng(N)
    D, F = W.random_instance(rng, N, 0, 20)
    p = rng.permutation(N).astype(np.int32)
    r = N // 2
    dE = orc.delta_row(D, F, p, r)
    beta = scale / max(1.0, float(np.std(dE)))
    M = 300_000
    counts = orc.sample_choices(dE, beta, 2, r, 0, 1, 0, M)
    probs = softmax64(dE, beta)
    assert chi2_pvalue(counts, probs) > 1e-3
    # a wrong sign of beta would be rejected decisively
    assert chi2_pvalue(counts, softmax64(-dE, beta)) < 1e-12


def sweep_kernel(D, F, beta):
    """Exact transition matrix of one sweep (updates of locations 0..N-1 in
    order) on all N! states, each update drawing among N candidates (stay
    included) with Eq. 5, energies from Eq. 1 in float64."""
    N = D.shape[0]
    states = [tuple(q) for q in itertools.permutations(range(N))]
    index = {s: i for i, s in enumerate(states)}
    Di, Fi = D.astype(np.int64), F.astype(np.int64)
    E = np.array([int(np.sum(Di * Fi[np.ix_(s, s)])) for s in states], dtype=np.float64)
    n = len(states)
    K = np.eye(n)
    for r in range(N):
        Kr = np.zeros((n, n))
        for a, s in enumerate(states):
            targets = []
            for k in range(N):
                q = list(s)
                q[r], q[k] = q[k], q[r]
                targets.append(index[tuple(q)])
            w = np.exp(-beta * (E[targets] - E[a]))
            w /= w.sum()
            for t, wt in zip(targets, w):
                Kr[a, t] += wt
        K = K @ Kr
    vals, vecs = np.linalg.eig(K.T)
    pi = np.real(vecs[:, np.argmin(np.abs(vals - 1))])
    pi /= pi.sum()
    boltz = np.exp(-beta * (E - E.min()))
    boltz /= boltz.sum()
    return states, E, pi, boltz


def test_two_location_law_is_boltzmann():
    rng = np.random.default_rng(0)
    D, F = W.random_instance(rng, 2, 1, 9)
    _, _, pi, boltz = sweep_kernel(D, F, 0.3)
    assert np.allclose(pi, boltz, atol=1e-12)


@pytest.mark.parametrize("N,beta,seed", [(2, 0.2, 13), (3, 0.2, 28), (4, 0.1, 9)])
def test_stationary_law_of_the_sweep(orc, N, beta, seed):
    """Final states of many independent chains match the exact stationary
    vector of the one-sweep kernel; for N >= 3 that vector is not the
    Boltzmann law and a Boltzmann fit is rejected."""
    rng = np.random.default_rng(seed)
    D, F = W.random_instance(rng, N, 0, 9)
    states, E, pi, boltz = sweep_kernel(D, F, beta)
    tv = 0.5 * np.abs(pi - boltz).sum()
    R, T = 40_000, 24
    perms = W.random_perms(np.random.default_rng(1), R, N)
    res = orc.run(D, F, perms, np.full(T, beta, np.float32), seed=2)
    index = {s: i for i, s in enumerate(states)}
    counts = np.zeros(len(states), dtype=np.int64)
    for row in res.perm:
        counts[index[tuple(int(v) for v in row)]] += 1
    assert chi2_pvalue(counts, pi) > 1e-3
    if N >= 3:
        assert tv > 0.05
        assert chi2_pvalue(counts, boltz) < 1e-6
    else:
        assert tv < 1e-12


def test_run_uses_counter_layout(orc):
    """With beta = 0 every update of a run picks floor(u N) for
    u = Philox(seed; r, g, replica, instance) word 0 >> 8."""
    N, T, R = 7, 5, 3
    rng = np.random.default_rng(9)
    D, F = W.random_instance(rng, N, 0, 9)
    perms = W.random_perms(rng, R, N)
    res = orc.run(D, F, perms, np.zeros(T, np.float32), seed=0xABCDEF0123, sweep_offset=40,
                  rep_ids=[5, 9, 2], inst_id=3, record_choices=True)
    for row, rep in enumerate([5, 9, 2]):
        for t in range(T):
            for r in range(N):
                u = orc.uniform24(0xABCDEF0123, r, 40 + t, rep, 3)
                assert res.choices[row, t, r] == (u * N) >> 24
