"""Seeded synthetic workloads for the symmetric QAP p-dit sweep.

This module only draws inputs: distance matrices D, flow matrices F, initial
permutations and inverse-temperature schedules.  It holds none of the
method's arithmetic (no energies, influences, swap deltas or sampling), so
both the GPU path and the CPU oracle can consume what it produces.

The paper measures on QAPLIB instances (Results, "Performance"; Table 1),
which are not available here; these generators stand in for them with the
structures QAPLIB's families have: grid-Manhattan distances with sparse
small-integer flows, uniform dense integer matrices, and Euclidean distances
with 0/1 flows.  Every generator is driven by numpy's PCG64
(``numpy.random.default_rng``).

Conventions (all configurations):
  * symmetric matrices are drawn on the strict upper triangle in row-major
    order, mirrored, and given a zero diagonal (the paper's "physical case"
    for Eq. 4);
  * instance seed 0, initial-permutation seed 1 (``rng.permutation(N)`` once
    per replica, in replica order), Philox seed 2;
  * inverse-temperature schedules are float32 arrays, one value per sweep.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

INSTANCE_SEED = 0
PERM_SEED = 1
PHILOX_SEED = 2


@dataclass
class Instance:
    """One QAP instance with its replicas' initial state and schedule."""

    name: str
    D: np.ndarray          # int32 [N, N], symmetric
    F: np.ndarray          # int32 [N, N], symmetric
    perms: np.ndarray      # int32 [R, N], each row a permutation of 0..N-1
    beta: np.ndarray       # float32 [T]
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return int(self.D.shape[0])

    @property
    def R(self) -> int:
        return int(self.perms.shape[0])

    @property
    def T(self) -> int:
        return int(self.beta.shape[0])


# ---------------------------------------------------------------------------
# matrix builders
# ---------------------------------------------------------------------------
def _mirror_upper(N: int, upper_values: np.ndarray) -> np.ndarray:
    """Place ``upper_values`` (length N(N-1)/2, row-major i<j) in a symmetric
    int32 matrix with zero diagonal."""
    M = np.zeros((N, N), dtype=np.int64)
    iu = np.triu_indices(N, k=1)
    M[iu] = upper_values
    M = M + M.T
    return M.astype(np.int32)


def sym_uniform(rng: np.random.Generator, N: int, lo: int, hi: int,
                zero_frac: float = 0.0) -> np.ndarray:
    """Symmetric, zero diagonal, upper triangle uniform integers in [lo, hi];
    then (if ``zero_frac`` > 0) each upper entry is zeroed with that
    probability."""
    m = N * (N - 1) // 2
    vals = rng.integers(lo, hi + 1, size=m, dtype=np.int64)
    if zero_frac > 0.0:
        keep = rng.random(m) >= zero_frac
        vals = vals * keep
    return _mirror_upper(N, vals)


def sym_bernoulli_values(rng: np.random.Generator, N: int, density: float,
                         lo: int, hi: int) -> np.ndarray:
    """Symmetric, zero diagonal; each upper entry is nonzero with probability
    ``density`` and then uniform in [lo, hi]."""
    m = N * (N - 1) // 2
    mask = rng.random(m) < density
    vals = rng.integers(lo, hi + 1, size=m, dtype=np.int64)
    return _mirror_upper(N, vals * mask)


def grid_manhattan(N: int, cols: int) -> np.ndarray:
    """Manhattan distances between the first N cells (row-major) of a grid
    with ``cols`` columns: location i sits at (i // cols, i % cols)."""
    idx = np.arange(N)
    y, x = idx // cols, idx % cols
    Dm = np.abs(y[:, None] - y[None, :]) + np.abs(x[:, None] - x[None, :])
    return Dm.astype(np.int32)


def euclid_points(rng: np.random.Generator, N: int, side: float = 100.0) -> np.ndarray:
    """Rounded Euclidean distances of N uniform points in [0, side]^2."""
    pts = rng.random((N, 2)) * side
    diff = pts[:, None, :] - pts[None, :, :]
    Dm = np.rint(np.sqrt((diff ** 2).sum(-1)))
    np.fill_diagonal(Dm, 0.0)
    return Dm.astype(np.int32)


def random_perms(rng: np.random.Generator, R: int, N: int) -> np.ndarray:
    return np.stack([rng.permutation(N) for _ in range(R)]).astype(np.int32)


# ---------------------------------------------------------------------------
# schedules
# ---------------------------------------------------------------------------
def beta_linear(b0: float, b1: float, T: int) -> np.ndarray:
    if T == 1:
        return np.array([b0], dtype=np.float32)
    t = np.arange(T, dtype=np.float64)
    return (b0 + (b1 - b0) * t / (T - 1)).astype(np.float32)


def beta_geometric(b0: float, b1: float, T: int) -> np.ndarray:
    if T == 1:
        return np.array([b0], dtype=np.float32)
    t = np.arange(T, dtype=np.float64)
    return (b0 * (b1 / b0) ** (t / (T - 1))).astype(np.float32)


def energy_scale(D: np.ndarray, F: np.ndarray) -> float:
    """A size scale for swap energy changes computed from data statistics
    only: 4 sqrt(N-2) sd(D_offdiag) sd(F_offdiag), which is the RMS change of
    a random transposition when the off-diagonal entries are independent.
    Used to put the annealing schedules of different instances on a common
    footing (beta * scale from 0.5 to 2000)."""
    N = D.shape[0]
    off = ~np.eye(N, dtype=bool)
    sd_d = float(np.std(D[off].astype(np.float64)))
    sd_f = float(np.std(F[off].astype(np.float64)))
    s = 4.0 * math.sqrt(max(N - 2, 1)) * sd_d * sd_f
    return s if s > 0 else 1.0


# ---------------------------------------------------------------------------
# the five workload configurations
# ---------------------------------------------------------------------------
def config_n12(R: int = 1, T: int = 1000) -> Instance:
    """N=12: D = Manhattan distances on a 3x4 grid; F symmetric, zero
    diagonal, off-diagonal uniform in [0, 9] with half of them zeroed
    (instance seed 0); linear beta 0.01 -> 2.0."""
    N = 12
    rng = np.random.default_rng(INSTANCE_SEED)
    D = grid_manhattan(N, 4)
    F = sym_uniform(rng, N, 0, 9, zero_frac=0.5)
    perms = random_perms(np.random.default_rng(PERM_SEED), R, N)
    return Instance("qap_n12_grid", D, F, perms, beta_linear(0.01, 2.0, T),
                    {"beta_rule": "linear 0.01->2.0"})


def config_n64(R: int = 1024, T: int = 10_000) -> Instance:
    """N=64: D and F symmetric, zero diagonal, uniform integers in [0, 99];
    geometric beta 0.001 -> 1.0."""
    N = 64
    rng = np.random.default_rng(INSTANCE_SEED)
    D = sym_uniform(rng, N, 0, 99)
    F = sym_uniform(rng, N, 0, 99)
    perms = random_perms(np.random.default_rng(PERM_SEED), R, N)
    return Instance("qap_n64_uniform99", D, F, perms, beta_geometric(1e-3, 1.0, T),
                    {"beta_rule": "geometric 0.001->1.0"})


def config_uneven(n_inst: int = 256, R: int = 64, T: int = 2000,
                  nmin: int = 20, nmax: int = 150) -> list[Instance]:
    """Uneven batch: instance k has N_k uniform in [nmin, nmax].  Even k:
    grid-Manhattan D (ceil(sqrt N) columns, first N cells) with flows that
    are nonzero with probability 0.3 and then uniform in [1, 9]; odd k:
    uniform [0, 99] D and F.  Geometric beta 0.5/s_k -> 2000/s_k."""
    rng = np.random.default_rng(INSTANCE_SEED)
    prng = np.random.default_rng(PERM_SEED)
    Ns = rng.integers(nmin, nmax + 1, size=n_inst)
    out = []
    for k in range(n_inst):
        N = int(Ns[k])
        if k % 2 == 0:
            D = grid_manhattan(N, int(math.ceil(math.sqrt(N))))
            F = sym_bernoulli_values(rng, N, 0.3, 1, 9)
            kind = "grid30"
        else:
            D = sym_uniform(rng, N, 0, 99)
            F = sym_uniform(rng, N, 0, 99)
            kind = "uniform99"
        s = energy_scale(D, F)
        perms = random_perms(prng, R, N)
        out.append(Instance(f"uneven_{k}_{kind}_n{N}", D, F, perms,
                            beta_geometric(0.5 / s, 2000.0 / s, T),
                            {"beta_rule": "geometric 0.5/s->2000/s", "scale": s}))
    return out


def config_n256(R: int = 512, T: int = 100_000) -> Instance:
    """N=256: D = rounded Euclidean distances of 256 uniform points in
    [0,100]^2; F symmetric 0/1 with density 0.1 and zero diagonal;
    geometric beta 0.5/s -> 2000/s."""
    N = 256
    rng = np.random.default_rng(INSTANCE_SEED)
    D = euclid_points(rng, N)
    F = sym_bernoulli_values(rng, N, 0.1, 1, 1)
    s = energy_scale(D, F)
    perms = random_perms(np.random.default_rng(PERM_SEED), R, N)
    return Instance("qap_n256_euclid", D, F, perms, beta_geometric(0.5 / s, 2000.0 / s, T),
                    {"beta_rule": "geometric 0.5/s->2000/s", "scale": s})


def clique_flows(N: int, members) -> np.ndarray:
    """F[a][b] = 1 for two distinct facilities of the clique, 0 otherwise."""
    c = np.zeros(N, dtype=np.int32)
    c[np.asarray(members)] = 1
    F = np.outer(c, c).astype(np.int32)
    np.fill_diagonal(F, 0)
    return F


def config_clique256(R: int = 512, T: int = 10_000) -> Instance:
    """N=256 with clique flows, a synthetic stand-in for tai256c (Methods):
    D = Manhattan distances on a 16 x 16 grid, F = 1 between any two of the
    first 92 facilities and 0 otherwise; geometric beta 0.5/s -> 2000/s."""
    N = 256
    D = grid_manhattan(N, 16)
    F = clique_flows(N, np.arange(92))
    s = energy_scale(D, F)
    perms = random_perms(np.random.default_rng(PERM_SEED), R, N)
    return Instance("qap_n256_clique92_grid16", D, F, perms, beta_geometric(0.5 / s, 2000.0 / s, T),
                    {"beta_rule": "geometric 0.5/s->2000/s", "scale": s, "clique": 92})


def config_n512(R: int = 256, T: int = 20_000) -> Instance:
    """N=512: D and F symmetric uniform integers in [0, 10^4] with 20% of
    entries zeroed; geometric beta 0.5/s -> 2000/s."""
    N = 512
    rng = np.random.default_rng(INSTANCE_SEED)
    D = sym_uniform(rng, N, 0, 10_000, zero_frac=0.2)
    F = sym_uniform(rng, N, 0, 10_000, zero_frac=0.2)
    s = energy_scale(D, F)
    perms = random_perms(np.random.default_rng(PERM_SEED), R, N)
    return Instance("qap_n512_uniform1e4", D, F, perms, beta_geometric(0.5 / s, 2000.0 / s, T),
                    {"beta_rule": "geometric 0.5/s->2000/s", "scale": s})


def random_instance(rng: np.random.Generator, N: int, lo: int = 0, hi: int = 9,
                    symmetric: bool = True, zero_diag: bool = True) -> tuple[np.ndarray, np.ndarray]:
    """Small random test instance; with ``zero_diag=False`` the diagonals are
    drawn too, and with ``symmetric=False`` every entry is independent."""
    if symmetric:
        D = sym_uniform(rng, N, lo, hi).astype(np.int64)
        F = sym_uniform(rng, N, lo, hi).astype(np.int64)
        if not zero_diag:
            D[np.diag_indices(N)] = rng.integers(lo, hi + 1, size=N)
            F[np.diag_indices(N)] = rng.integers(lo, hi + 1, size=N)
    else:
        D = rng.integers(lo, hi + 1, size=(N, N))
        F = rng.integers(lo, hi + 1, size=(N, N))
        if zero_diag:
            np.fill_diagonal(D, 0)
            np.fill_diagonal(F, 0)
    return D.astype(np.int32), F.astype(np.int32)
