"""Pins of the oracle's sweep engine: the incrementally kept influence and
energy against recomputation, determinism and resume, replica
independence, and that the annealer reaches brute-force optima."""
import numpy as np
import pytest

from paper_2605_24408_amd import workloads as W
from test_oracle_equations import energy_trace


@pytest.mark.parametrize("N,sym_diag", [(5, False), (9, True), (16, False)])
def test_paranoid_run_keeps_influence_exact(orc, N, sym_diag):
    """A hot run with many accepted swaps: after every sweep the kept
    influence equals Eq. 2 recomputed and the kept energy equals Eq. 1."""
    rng = np.random.default_rng(N)
    D, F = W.random_instance(rng, N, -30, 99, symmetric=True, zero_diag=sym_diag)
    perms = W.random_perms(rng, 3, N)
    res = orc.run(D, F, perms, np.full(40, 1e-4, np.float32), seed=5, paranoid=True)
    assert res.counters[:, 1].sum() > 50
    for k in range(3):
        assert res.E[k] == energy_trace(D, F, res.perm[k])
        assert res.E_best[k] == energy_trace(D, F, res.perm_best[k])
        assert res.E_best[k] <= res.E[k]
        assert sorted(res.perm[k]) == list(range(N))


def test_asymmetric_data_paranoid(orc):
    """Eq. 2 and Eq. 3 hold for asymmetric data too; the incremental update
    keeps them exact."""
    rng = np.random.default_rng(77)
    D, F = W.random_instance(rng, 7, 0, 50, symmetric=False, zero_diag=False)
    perms = W.random_perms(rng, 2, 7)
    res = orc.run(D, F, perms, np.full(30, 0.01, np.float32), seed=1, paranoid=True)
    for k in range(2):
        assert res.E[k] == energy_trace(D, F, res.perm[k])


def test_resume_equals_uninterrupted(orc):
    inst = W.config_n12(R=4, T=300)
    full = orc.run(inst.D, inst.F, inst.perms, inst.beta, seed=2)
    a = orc.run(inst.D, inst.F, inst.perms, inst.beta[:120], seed=2)
    b = orc.run(inst.D, inst.F, a.perm, inst.beta[120:], seed=2, sweep_offset=120,
                E_best=a.E_best, perm_best=a.perm_best)
    assert np.array_equal(full.perm, b.perm)
    assert np.array_equal(full.E, b.E)
    assert np.array_equal(full.E_best, b.E_best)
    assert np.array_equal(full.perm_best, b.perm_best)
    assert np.array_equal(full.counters[:, :2], a.counters[:, :2] + b.counters[:, :2])


def test_replica_does_not_depend_on_batch(orc):
    inst = W.config_n12(R=6, T=80)
    batch = orc.run(inst.D, inst.F, inst.perms, inst.beta, seed=2)
    for k in (0, 3, 5):
        one = orc.run(inst.D, inst.F, inst.perms[k:k + 1], inst.beta, seed=2, rep_ids=[k])
        assert np.array_equal(one.perm[0], batch.perm[k])
        assert one.E_best[0] == batch.E_best[k]


def test_bad_permutation_rejected(orc):
    inst = W.config_n12(R=1, T=2)
    p = inst.perms.copy()
    p[0, 3] = p[0, 4]
    with pytest.raises(RuntimeError):
        orc.run(inst.D, inst.F, p, inst.beta, seed=2)


@pytest.mark.parametrize("N", [6, 7, 8])
def test_annealing_reaches_brute_force_optimum(orc, N):
    rng = np.random.default_rng(300 + N)
    D, F = W.random_instance(rng, N, 0, 20)
    opt, _ = orc.brute_min(D, F)
    perms = W.random_perms(rng, 8, N)
    s = W.energy_scale(D, F)
    res = orc.run(D, F, perms, W.beta_geometric(0.5 / s, 50.0 / s, 400), seed=2)
    assert res.E_best.min() == opt
    assert (res.E_best >= opt).all()


def test_n12_workload_reaches_exact_optimum(orc):
    """The N=12 grid workload, 16 replicas of its schedule: the best energy
    found is the exhaustively computed optimum."""
    import json
    import os
    from conftest import GOLDEN
    g = json.load(open(os.path.join(GOLDEN, "qap_n12_optimum.json")))
    inst = W.config_n12(R=16)
    res = orc.run(inst.D, inst.F, inst.perms, inst.beta, seed=2)
    assert (res.E_best >= g["optimum"]).all()
    assert res.E_best.min() == g["optimum"]
