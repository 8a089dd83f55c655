"""Seeded synthetic charge sets (inputs only; none of the method's arithmetic).

Both the GPU path's tests and the oracle's tests draw their inputs here, so the
two sides see bit-identical positions and charges.  Generator: NumPy PCG64
(``numpy.random.default_rng(seed)``); positions are drawn first, then charges.

Workloads (sizes of the Coulomb-sum problems the library is measured on):
  * ``uniform_pm1``   : x ~ U[0,1)^3, q = +-1 with exactly floor(n/2) of +1 and
                        the rest -1, randomly permuted (net zero for even n).
  * ``uniform_gauss`` : x ~ U[0,1)^3, q ~ N(0,1) minus its FP64 mean.
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
