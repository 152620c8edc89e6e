"""Pins of the clique-flow specialisation (Methods, "CPU-PIM Algorithm",
tai256c): with F[a][b] = 1 for two distinct facilities of a clique C and 0
otherwise, and D symmetric with a zero diagonal, Eq. 1 depends only on the
set S of locations holding clique facilities, and with g(x) = sum_{j in S}
D[x][j] the energy change of exchanging locations r and s is

    0                              when r and s are in the same class,
    2 (g(s) - g(r) - D[r][s])      when r is in S and s is not,
    2 (g(r) - g(s) - D[r][s])      when s is in S and r is not.

The GPU's clique kernel evaluates exactly this; here it is checked against
Eq. 3 (the oracle's rows, pinned against full recomputation) and the energy
against Eq. 1."""
import numpy as np
import pytest

import oracle
from paper_2605_24408_amd import workloads as W


def clique_F(N, members):
    c = np.zeros(N, np.int64)
    c[members] = 1
    F = np.outer(c, c)
    np.fill_diagonal(F, 0)
    return F


@pytest.mark.parametrize("N,m", [(6, 2), (12, 5), (40, 17), (64, 1), (64, 63), (90, 45)])
def test_closed_form_equals_eq3(N, m):
    rng = np.random.default_rng(N + m)
    D = W.sym_uniform(rng, N, 0, 50).astype(np.int64)
    members = rng.permutation(N)[:m]
    F = clique_F(N, members)
    isc = np.zeros(N, bool)
    isc[members] = True
    for _ in range(3):
        p = rng.permutation(N).astype(np.int32)
        S = isc[p]  # location x holds a clique facility
        g = D[:, S].sum(axis=1)
        E = int(D[np.ix_(S, S)].sum())
        assert E == oracle.energy(D, F, p)
        for r in range(N):
            want = oracle.delta_row(D, F, p, r)
            got = np.zeros(N, np.int64)
            for s in range(N):
                if S[r] and not S[s]:
                    got[s] = 2 * (g[s] - g[r] - D[r, s])
                elif S[s] and not S[r]:
                    got[s] = 2 * (g[r] - g[s] - D[r, s])
            assert np.array_equal(got, want), r


def test_g_update_after_a_cross_class_exchange():
    """After exchanging r in S with s outside, g'(x) = g(x) - D[x][r] + D[x][s]."""
    rng = np.random.default_rng(3)
    N = 30
    D = W.sym_uniform(rng, N, 0, 40).astype(np.int64)
    members = np.arange(11)
    isc = np.zeros(N, bool)
    isc[members] = True
    p = rng.permutation(N).astype(np.int32)
    S = isc[p]
    r = int(np.nonzero(S)[0][0])
    s = int(np.nonzero(~S)[0][0])
    g = D[:, S].sum(axis=1)
    q = p.copy()
    q[r], q[s] = q[s], q[r]
    S2 = isc[q]
    assert np.array_equal(D[:, S2].sum(axis=1), g - D[:, r] + D[:, s])
