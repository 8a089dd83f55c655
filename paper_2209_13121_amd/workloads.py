"""Seeded synthetic charge sets (inputs only; none of the method's arithmetic).

Both the GPU path's tests and the oracle's tests draw their inputs here, so the
two sides see bit-identical positions and charges.  Generator: NumPy PCG64
(``numpy.random.default_rng(seed)``); positions are drawn first, then charges.

Workloads (sizes of the Coulomb-sum problems the library is measured on):
  * ``uniform_pm1``   : x ~ U[0,1)^3, q = +-1 with exactly floor(n/2) of +1 and
                        the rest -1, randomly permuted (net zero for even n).
  * ``uniform_gauss`` : x ~ U[0,1)^3, q ~ N(0,1) minus its FP64 mean.
  * ``molecular_clusters`` : three-site clusters (charges -0.834, +0.417,
                        +0.417; bond 0.0957 nm; angle 104.5 deg; orientation
                        uniform on SO(3) from a random unit quaternion) whose
                        first sites are drawn by rejection from the density
                        rho0 (1 + 3 max_k exp(-|x - c_k|^2 / (2 sigma^2))),
                        rho0 = 100 sites/nm^3, 16 blob centres uniform in the
                        cube, sigma = side/16; the cube side is set so that
                        the expected cluster count is the one asked for.
"""
from dataclasses import dataclass

import numpy as np


def uniform_pm1(n: int, seed: int):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    q = np.empty(n)
    q[: n // 2] = 1.0
    q[n // 2:] = -1.0
    rng.shuffle(q)
    return pos, q


def uniform_gauss(n: int, seed: int):
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    q = rng.standard_normal(n)
    q -= q.mean()
    return pos, q


CLUSTER_Q = (-0.834, 0.417, 0.417)
CLUSTER_BOND_NM = 0.0957
CLUSTER_ANGLE_DEG = 104.5


def molecular_clusters(n_clusters: int, seed: int, rho0: float = 100.0, blobs: int = 16,
                       contrast: float = 3.0):
    """Positions (nm, 3 n_clusters x 3) and charges of n_clusters three-site
    clusters; returns (pos, q, side) with side the cube edge the density was
    laid out on (sites may stick out of [0, side]^3 by up to one bond)."""
    rng = np.random.default_rng(seed)
    centres = rng.random((blobs, 3))  # in units of the cube side
    sig = 1.0 / 16.0

    def density_factor(x):  # rho / rho0 at unit-cube coordinates x, in chunks
        out = np.empty(len(x))
        for a in range(0, len(x), 1 << 18):
            d2 = ((x[a:a + (1 << 18), None, :] - centres[None, :, :]) ** 2).sum(axis=2)
            out[a:a + (1 << 18)] = 1.0 + contrast * np.exp(-d2.min(axis=1) / (2 * sig * sig))
        return out

    mean_f = density_factor(rng.random((200_000, 3))).mean()
    side = (3.0 * n_clusters / (rho0 * mean_f)) ** (1.0 / 3.0)
    first = np.empty((0, 3))
    while len(first) < n_clusters:
        cand = rng.random((max(2 * (n_clusters - len(first)), 1024), 3))
        keep = rng.random(len(cand)) * (1.0 + contrast) < density_factor(cand)
        first = np.concatenate([first, cand[keep]])
    first = first[:n_clusters] * side
    # random unit quaternions -> rotation matrices (uniform on SO(3))
    qt = rng.standard_normal((n_clusters, 4))
    qt /= np.linalg.norm(qt, axis=1, keepdims=True)
    w, x, y, z = qt.T
    R = np.stack([np.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
                  np.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
                  np.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)],
                 axis=1)
    half = np.deg2rad(CLUSTER_ANGLE_DEG) / 2.0
    body = CLUSTER_BOND_NM * np.array([[np.sin(half), 0.0, np.cos(half)],
                                       [-np.sin(half), 0.0, np.cos(half)]])
    sites = np.empty((n_clusters, 3, 3))
    sites[:, 0] = first
    sites[:, 1:] = first[:, None, :] + np.einsum("cij,sj->csi", R, body)
    q = np.tile(np.array(CLUSTER_Q), n_clusters)
    return sites.reshape(-1, 3), q, side


@dataclass(frozen=True)
class Workload:
    name: str
    n: int
    depth: int
    p: int
    charges: str  # "pm1" or "gauss"
    seed: int

    def make(self):
        gen = uniform_pm1 if self.charges == "pm1" else uniform_gauss
        return gen(self.n, self.seed)


# Small case: N = 4096 point charges, unit cube, uniform octree of depth 3, p = 4.
SMALL = Workload("uniform-pm1-n4096-depth3-p4", 4096, 3, 4, "pm1", 1001)
# Headline case: N = 2^20 Gaussian charges, unit cube, depth 6, p = 8.
HEADLINE = Workload("uniform-gauss-n1048576-depth6-p8", 1 << 20, 6, 8, "gauss", 1002)
# Differentiation case: N = 2^19 +-1 charges, depth 6, p = 8.
ADJOINT = Workload("uniform-pm1-n524288-depth6-p8", 1 << 19, 6, 8, "pm1", 1004)


@dataclass(frozen=True)
class ClusterWorkload:
    name: str
    n_clusters: int
    leaf_max: int
    max_depth: int
    p: int
    seed: int

    @property
    def n(self):
        return 3 * self.n_clusters

    def make(self):
        pos, q, _ = molecular_clusters(self.n_clusters, self.seed)
        return pos, q


# Adaptive case: 10^6 three-site clusters (3e6 sites), leaves of at most 64
# sites, p = 10, mixed precision.
CLUSTERS = ClusterWorkload("clusters-n3000000-leaf64-p10", 1_000_000, 64, 7, 10, 1003)


def batched_systems(n_systems: int, seed: int, n_min: int = 1000, n_max: int = 65536,
                    grid: int = 8):
    """A batch of independent systems: N_k = round(exp(U[ln n_min, ln n_max]))
    rounded up to even, positions uniform in the system's own unit cube, the
    k-th cube at cell (k % g, (k // g) % g, k // g^2) of a g^3 grid (root cube
    [0, g]^3, so the systems are the boxes of level log2(g)), +-1 charges
    with exactly N_k / 2 of each sign, shuffled.  Returns (pos, q, counts)."""
    assert n_systems <= grid ** 3
    rng = np.random.default_rng(seed)
    counts = np.round(np.exp(rng.uniform(np.log(n_min), np.log(n_max), n_systems))).astype(np.int64)
    counts += counts % 2
    pos, q = [], []
    for k, nk in enumerate(counts):
        cell = np.array([k % grid, (k // grid) % grid, k // (grid * grid)], dtype=float)
        pos.append(cell + rng.random((nk, 3)))
        qk = np.empty(nk)
        qk[: nk // 2] = 1.0
        qk[nk // 2:] = -1.0
        rng.shuffle(qk)
        q.append(qk)
    return np.concatenate(pos), np.concatenate(q), counts


@dataclass(frozen=True)
class BatchWorkload:
    name: str
    n_systems: int
    leaf_max: int
    max_depth: int
    batch_level: int
    p: int
    seed: int

    def make(self):
        return batched_systems(self.n_systems, self.seed, grid=1 << self.batch_level)


# Batched case: 256 systems of 10^3 .. 2^16 +-1 charges (log-uniform, about
# 4e6 in all), each in its own unit cell of an 8^3 grid, adaptive leaves of at
# most 64, p = 6.
BATCH = BatchWorkload("batch256-n1e3to65536-leaf64-p6", 256, 64, 7, 3, 6, 1005)
