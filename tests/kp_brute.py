"""Basis-free brute force of the FMM result (pin for the oracle's operators).

For a target at x (leaf ancestor t at level l, centre c_t) and a source at y in
a box s of t's interaction list (centre c_s), the FMM with full truncation
replaces 1/|x - y| by

    K_p(u, v; d) = sum_{a<=p, b<=p} [s^a t^b] |d + s u - t v|^{-1}
                 = sum_{a<=p, b<=p} [s^a t^b] (D (1 + X(s, t)))^{-1/2},
    u = x - c_t,  v = y - c_s,  d = c_t - c_s,  D = |d|^2,
    D X = 2 s d.u - 2 t d.v + s^2 u.u - 2 s t u.v + t^2 v.v,

i.e. the part of the two-variable Taylor series of 1/|d + u - v| of degree
<= p in u and <= p in v (Greengard 1988, ch. 3; Cheng, Greengard & Rokhlin
1999).  The binomial series (1+X)^{-1/2} = sum_k C(-1/2, k) X^k is evaluated
in truncated two-variable power-series arithmetic (Griewank & Walther,
"Evaluating Derivatives", 2nd ed., ch. 13).  X has no constant term, so
k <= 2p suffices for every retained (a, b).

Gradients with respect to x use the complex-step derivative (Squire & Trapp,
SIAM Rev. 40:110 (1998)): the same series evaluated at u + i h e_a with the
analytic continuation u.u, so Im K / h is exact to rounding for tiny h.

None of the spherical-harmonic formulas of the oracle are used here.
"""
import numpy as np


def _binom_mhalf(kmax):
    c = np.empty(kmax + 1)
    c[0] = 1.0
    for k in range(1, kmax + 1):
        c[k] = c[k - 1] * (-0.5 - (k - 1)) / k
    return c


def kp(u, v, d, p):
    """K_p for arrays u, v, d of shape (m, 3) (u may be complex)."""
    u = np.asarray(u)
    v = np.asarray(v, dtype=float)
    d = np.asarray(d, dtype=float)
    m = len(d)
    dt = np.result_type(u.dtype, np.float64)
    D = np.einsum("ij,ij->i", d, d)
    A = 2.0 * np.einsum("ij,ij->i", d, u) / D
    B = -2.0 * np.einsum("ij,ij->i", d, v) / D
    C = np.einsum("ij,ij->i", u, u) / D
    E = -2.0 * np.einsum("ij,ij->i", u, v) / D
    F = np.einsum("ij,ij->i", v, v) / D
    coef = _binom_mhalf(2 * p)
    P = np.zeros((m, p + 1, p + 1), dtype=dt)  # X^k, truncated at degree p in s and in t
    P[:, 0, 0] = 1.0
    S = coef[0] * P.copy()
    for k in range(1, 2 * p + 1):
        Q = np.zeros_like(P)
        Q[:, 1:, :] += A[:, None, None] * P[:, :-1, :]
        Q[:, :, 1:] += B[:, None, None] * P[:, :, :-1]
        Q[:, 2:, :] += C[:, None, None] * P[:, :-2, :]
        Q[:, 1:, 1:] += E[:, None, None] * P[:, :-1, :-1]
        Q[:, :, 2:] += F[:, None, None] * P[:, :, :-2]
        P = Q
        S += coef[k] * P
    return S.sum(axis=(1, 2)) / np.sqrt(D)


def kp_with_grad(u, v, d, p, h=1e-30):
    """K_p and its gradient with respect to u (complex step)."""
    u = np.asarray(u, dtype=float)
    val = np.real(kp(u.astype(complex), v, d, p))
    g = np.empty_like(u)
    for a in range(3):
        du = u.astype(complex)
        du[:, a] += 1j * h
        g[:, a] = np.imag(kp(du, v, d, p)) / h
    return val, g


def fmm_brute(pos, q, depth, p, lo=(0.0, 0.0, 0.0), side=1.0):
    """phi and grad phi of the FMM result at every particle, from the
    definition above (O(N^2) pairs; tiny inputs only)."""
    pos = np.asarray(pos, dtype=float)
    q = np.asarray(q, dtype=float)
    lo = np.asarray(lo, dtype=float)
    n = len(q)
    L = depth
    nb = 1 << L
    cell = np.clip(np.floor((pos - lo) / side * nb), 0, nb - 1).astype(np.int64)
    phi = np.zeros(n)
    grad = np.zeros((n, 3))
    for i in range(n):
        others = np.arange(n) != i
        # near field: leaves within Chebyshev distance 1
        near = others & (np.abs(cell - cell[i]).max(axis=1) <= 1)
        dx = pos[i] - pos[near]
        r = np.sqrt((dx * dx).sum(axis=1))
        phi[i] += (q[near] / r).sum()
        grad[i] -= ((q[near] / r**3)[:, None] * dx).sum(axis=0)
        # far field: for each level, sources whose level-l box is in the
        # interaction list of the target's level-l box
        for l in range(2, L + 1):
            sh = L - l
            bt = cell[i] >> sh
            bs = cell >> sh
            adj = np.abs(bs - bt).max(axis=1) <= 1
            padj = np.abs((bs >> 1) - (bt >> 1)).max(axis=1) <= 1
            far = others & padj & ~adj
            if not far.any():
                continue
            h = side / (1 << l)
            ct = lo + (bt + 0.5) * h
            cs = lo + (bs[far] + 0.5) * h
            u = np.broadcast_to(pos[i] - ct, (far.sum(), 3))
            v = pos[far] - cs
            d = ct - cs
            k, gk = kp_with_grad(u, v, d, p)
            phi[i] += (q[far] * k).sum()
            grad[i] += (q[far][:, None] * gk).sum(axis=0)
    return phi, grad
