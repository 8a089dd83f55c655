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


def kp_general(u, v, d, pa, pb):
    """The part of the Taylor series of 1/|d + s u - t v| of degree <= pa in s
    and <= pb in t, at s = t = 1 (u and d may be complex)."""
    u = np.asarray(u)
    v = np.asarray(v, dtype=float)
    d = np.asarray(d)
    m = len(d)
    dt = np.result_type(u.dtype, d.dtype, np.float64)
    D = np.einsum("ij,ij->i", d, d)
    A = 2.0 * np.einsum("ij,ij->i", d, u) / D
    B = -2.0 * np.einsum("ij,ij->i", d, v) / D
    C = np.einsum("ij,ij->i", u, u) / D
    E = -2.0 * np.einsum("ij,ij->i", u, v) / D
    F = np.einsum("ij,ij->i", v, v) / D
    coef = _binom_mhalf(pa + pb)
    P = np.zeros((m, pa + 1, pb + 1), dtype=dt)
    P[:, 0, 0] = 1.0
    S = coef[0] * P.copy()
    for k in range(1, pa + pb + 1):
        Q = np.zeros_like(P)
        if pa >= 1:
            Q[:, 1:, :] += A[:, None, None] * P[:, :-1, :]
        if pb >= 1:
            Q[:, :, 1:] += B[:, None, None] * P[:, :, :-1]
        if pa >= 2:
            Q[:, 2:, :] += C[:, None, None] * P[:, :-2, :]
        if pa >= 1 and pb >= 1:
            Q[:, 1:, 1:] += E[:, None, None] * P[:, :-1, :-1]
        if pb >= 2:
            Q[:, :, 2:] += F[:, None, None] * P[:, :, :-2]
        P = Q
        S += coef[k] * P
    return S.sum(axis=(1, 2)) / np.sqrt(D)


def _adjacent(a, la, c, lc):
    """Closed cubes of boxes a (level la) and c (level lc >= la) touch; a, c
    integer cells of shape (m, 3) or (3,)."""
    s = lc - la
    lo = np.asarray(a) << s
    hi = (np.asarray(a) + 1) << s
    c = np.asarray(c)
    return np.all((c <= hi) & (c + 1 >= lo), axis=-1)


def fmm_adaptive_brute(pos, q, leaf_max, max_depth, p, lo=(0.0, 0.0, 0.0), side=1.0):
    """phi and grad phi of the adaptive-tree FMM at every particle, pair by
    pair (tiny inputs only).  The tree: a box with more than leaf_max
    particles is divided while its level is below max_depth.  A pair (i, j)
    is handled by exactly one operator, found by walking the two ancestor
    chains from the root (Cheng, Greengard & Rokhlin 1999, sec. 4):
      * the first level l at which both chains still have a box and the two
        boxes are not adjacent: M2L at level l, kernel K_p(x_i - c_A, x_j - c_B;
        c_A - c_B) (truncated at degree p in both displacements);
      * else, when i's leaf a is coarser: the first box B_m of j's chain below
        a's level that is not adjacent to a: M2P, the source displacement
        truncated at degree p, the target exact;
      * else, when j's leaf is coarser: the dual (P2L, the target displacement
        truncated, the source exact);
      * else (the leaves touch): the exact 1/r.
    Returns (phi, grad, counts) where counts tallies the pairs per operator."""
    pos = np.asarray(pos, dtype=float)
    q = np.asarray(q, dtype=float)
    lo = np.asarray(lo, dtype=float)
    n = len(q)
    Lm = max_depth
    cell = np.clip(np.floor((pos - lo) / side * (1 << Lm)), 0, (1 << Lm) - 1).astype(np.int64)
    anc = np.stack([cell >> (Lm - l) for l in range(Lm + 1)])  # (levels, n, 3)
    leaf = np.full(n, Lm)
    for l in range(Lm, -1, -1):
        keys, inv, cnt = np.unique(anc[l], axis=0, return_inverse=True, return_counts=True)
        small = cnt[inv.ravel()] <= leaf_max
        leaf = np.where(small, l, leaf)  # the smallest such level wins (descending loop)
    phi = np.zeros(n)
    grad = np.zeros((n, 3))
    counts = {"p2p": 0, "m2l": 0, "m2p": 0, "p2l": 0}
    h = 1e-30

    def centre(c, l):
        return lo + (c + 0.5) * (side / (1 << l))

    for i in range(n):
        js = np.array([j for j in range(n) if j != i], dtype=np.int64)
        if len(js) == 0:
            continue
        la = leaf[i]
        lb = leaf[js]
        kind = np.full(len(js), -1)  # 0 p2p, 1 m2l, 2 m2p, 3 p2l
        lvl = np.full(len(js), -1)
        for l in range(Lm + 1):
            both = (l <= la) & (l <= lb) & (kind < 0)
            sep = both & ~_adjacent(anc[l, i], l, anc[l, js], l)
            kind[sep] = 1
            lvl[sep] = l
        # i's leaf coarser: descend j's chain
        for m in range(Lm + 1):
            sel = (kind < 0) & (la < lb) & (m > la) & (m <= lb)
            if sel.any():
                sep = sel & ~_adjacent(anc[la, i], la, anc[m, js], m)
                kind[sep] = 2
                lvl[sep] = m
            sel = (kind < 0) & (lb < la) & (m > lb) & (m <= la)
            if sel.any():
                sep = np.zeros(len(js), bool)
                for t in np.nonzero(sel)[0]:
                    sep[t] = not _adjacent(anc[lb[t], js[t]], lb[t], anc[m, i], m)
                kind[sep] = 3
                lvl[sep] = m
        kind[kind < 0] = 0
        assert np.all(lvl[kind == 1] >= 2)
        for k, name in enumerate(("p2p", "m2l", "m2p", "p2l")):
            counts[name] += int((kind == k).sum())
        x = pos[i]
        # exact near pairs
        s = js[kind == 0]
        dx = x - pos[s]
        r = np.sqrt((dx * dx).sum(axis=1))
        phi[i] += (q[s] / r).sum()
        grad[i] -= ((q[s] / r**3)[:, None] * dx).sum(axis=0)
        # M2L pairs, per level
        for l in range(2, Lm + 1):
            t = kind == 1
            t &= lvl == l
            if not t.any():
                continue
            s = js[t]
            ct = centre(anc[l, i], l)
            cs = centre(anc[l, s], l)
            u = np.broadcast_to(x - ct, (len(s), 3)).astype(complex)
            v = pos[s] - cs
            d = ct - cs
            val = np.real(kp_general(u, v, d, p, p))
            phi[i] += (q[s] * val).sum()
            for a in range(3):
                du = u.copy()
                du[:, a] += 1j * h
                grad[i, a] += (q[s] * np.imag(kp_general(du, v, d, p, p)) / h).sum()
        # M2P pairs: target exact (u = 0, d = x - c_B), source truncated
        t = kind == 2
        if t.any():
            s = js[t]
            cs = np.stack([centre(anc[lvl[k], js[k]], lvl[k]) for k in np.nonzero(t)[0]])
            v = pos[s] - cs
            d = (x - cs).astype(complex)
            u = np.zeros((len(s), 3), complex)
            phi[i] += (q[s] * np.real(kp_general(u, v, d, 0, p))).sum()
            for a in range(3):
                dd = d.copy()
                dd[:, a] += 1j * h
                grad[i, a] += (q[s] * np.imag(kp_general(u, v, dd, 0, p)) / h).sum()
        # P2L pairs: source exact (v = 0, d = c_A - y), target truncated
        t = kind == 3
        if t.any():
            s = js[t]
            ct = np.stack([centre(anc[lvl[k], i], lvl[k]) for k in np.nonzero(t)[0]])
            u = (x - ct).astype(complex)
            v = np.zeros((len(s), 3))
            d = ct - pos[s]
            phi[i] += (q[s] * np.real(kp_general(u, v, d, p, 0))).sum()
            for a in range(3):
                du = u.copy()
                du[:, a] += 1j * h
                grad[i, a] += (q[s] * np.imag(kp_general(du, v, d, p, 0)) / h).sum()
    return phi, grad, counts
