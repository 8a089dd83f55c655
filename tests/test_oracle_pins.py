"""Pins of the CPU oracle against facts fixed by mathematics (no GPU).

Each test checks the oracle against something other than its own formulas:
the basis-free truncated Taylor kernel, Legendre closed forms, exactness of
re-centring, invariants of the Coulomb sum, finite differences and the
tree's geometric rules.
"""
import math

import numpy as np
import pytest
from scipy.special import eval_legendre

import kp_brute
import oracle
from paper_2209_13121_amd import workloads as W


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# ---------------------------------------------------------------- brute force
def test_kp_with_zero_target_offset_is_legendre_series():
    """K_p(0, v; d) is the degree-<=p Legendre (multipole) series of 1/|d - v|."""
    rng = np.random.default_rng(1)
    for p in (0, 3, 8):
        v = rng.uniform(-0.5, 0.5, (20, 3))
        d = rng.uniform(-3, 3, (20, 3)) + np.array([4.0, 0, 0])
        k = kp_brute.kp(np.zeros((20, 3)), v, d, p)
        rv, rd = np.linalg.norm(v, axis=1), np.linalg.norm(d, axis=1)
        cosg = np.einsum("ij,ij->i", v, d) / (rv * rd)
        ref = sum(rv**n * eval_legendre(n, cosg) / rd ** (n + 1) for n in range(p + 1))
        assert np.max(np.abs(k - ref) / np.abs(ref)) < 1e-13


def test_kp_converges_to_inverse_distance():
    rng = np.random.default_rng(2)
    u = rng.uniform(-0.5, 0.5, (50, 3))
    v = rng.uniform(-0.5, 0.5, (50, 3))
    d = np.tile([2.0, 1.0, 0.0], (50, 1))
    exact = 1.0 / np.linalg.norm(d + u - v, axis=1)
    errs = [np.max(np.abs(kp_brute.kp(u, v, d, p) - exact) / exact) for p in (2, 4, 8, 12)]
    assert errs[-1] < 1e-6
    assert all(errs[i + 1] < errs[i] for i in range(len(errs) - 1))


# -------------------------------------------------------- the FMM as a whole
@pytest.mark.parametrize("depth,p", [(2, 0), (2, 1), (2, 4), (3, 2), (3, 4), (3, 8)])
def test_oracle_fmm_equals_truncated_taylor_definition(depth, p):
    """P2M, M2M, M2L, L2L, L2P and P2P together reproduce the basis-free
    definition of the truncated FMM, potentials and gradients."""
    pos, q = W.uniform_gauss(120, 10 + depth * 10 + p)
    phi_b, grad_b = kp_brute.fmm_brute(pos, q, depth, p)
    phi, force, energy = oracle.fmm(pos, q, depth, p)
    grad = -force / q[:, None]
    assert rel(phi, phi_b) < 1e-12
    assert rel(grad, grad_b) < 1e-12
    assert abs(energy - 0.5 * math.fsum(q * phi_b)) <= 1e-12 * abs(energy)


def test_oracle_fmm_nonunit_cube_equals_definition():
    pos, q = W.uniform_gauss(100, 77)
    lo, side = np.array([-3.0, 1.5, 0.25]), 2.5
    pos = lo + pos * side
    phi_b, grad_b = kp_brute.fmm_brute(pos, q, 3, 5, lo=lo, side=side)
    phi, force, _ = oracle.fmm(pos, q, 3, 5, lo=lo, side=side)
    assert rel(phi, phi_b) < 1e-12
    assert rel(-force / q[:, None], grad_b) < 1e-12


# ------------------------------------------------------------ single charge
def _legendre_series(q, y, c, x, p):
    ry = np.linalg.norm(y - c)
    rx = np.linalg.norm(x - c, axis=1)
    cosg = ((x - c) @ (y - c)) / (rx * ry)
    return q * sum(ry**n * eval_legendre(n, cosg) / rx ** (n + 1) for n in range(p + 1))


def test_single_charge_multipole_is_legendre_series():
    rng = np.random.default_rng(3)
    y = np.array([[0.1, -0.2, 0.15]])
    c1 = np.zeros(3)
    x = rng.uniform(-1, 1, (30, 3)) + np.array([2.0, 1.0, -1.5])
    for p in (0, 1, 4, 9):
        phi, _ = oracle.chain(oracle.CHAIN_M2P, p, y, [1.7], x, c1)
        ref = _legendre_series(1.7, y[0], c1, x, p)
        assert np.max(np.abs(phi - ref) / np.abs(ref)) < 1e-13


def test_multipole_truncation_obeys_error_bound():
    """|phi - phi_p| <= q/(r - a) (a/r)^{p+1} (Greengard 1988, ch. 3)."""
    rng = np.random.default_rng(4)
    y = np.array([[0.3, 0.2, -0.1]])
    a = np.linalg.norm(y)
    x = rng.normal(size=(40, 3))
    x = 1.5 * x / np.linalg.norm(x, axis=1)[:, None]
    r = np.linalg.norm(x, axis=1)
    exact = 1.0 / np.linalg.norm(x - y, axis=1)
    for p in (2, 5, 10):
        phi, _ = oracle.chain(oracle.CHAIN_M2P, p, y, [1.0], x, np.zeros(3))
        assert np.all(np.abs(phi - exact) <= 1.0 / (r - a) * (a / r) ** (p + 1) * (1 + 1e-12))


def test_m2m_is_exact_shift():
    """Shifting a single charge's multipole gives its multipole about the new
    centre: the Legendre series about c2."""
    rng = np.random.default_rng(5)
    y = np.array([[0.1, 0.05, -0.1]])
    c1 = np.array([0.125, -0.125, 0.125])
    c2 = np.zeros(3)
    x = rng.uniform(-1, 1, (25, 3)) + np.array([3.0, -2.0, 1.0])
    for p in (2, 6, 10):
        phi, _ = oracle.chain(oracle.CHAIN_M2M_M2P, p, y, [-0.8], x, c1, c2)
        ref = _legendre_series(-0.8, y[0], c2, x, p)
        assert np.max(np.abs(phi - ref) / np.abs(ref)) < 1e-12


def test_m2l_l2p_equals_truncated_kernel_with_gradient():
    rng = np.random.default_rng(6)
    src = rng.uniform(-0.5, 0.5, (4, 3))
    q = rng.normal(size=4)
    c1, c2 = np.zeros(3), np.array([2.0, -3.0, 1.0])
    x = c2 + rng.uniform(-0.5, 0.5, (15, 3))
    for p in (1, 4, 8):
        phi, grad = oracle.chain(oracle.CHAIN_M2L_L2P, p, src, q, x, c1, c2)
        ref = np.zeros(15)
        gref = np.zeros((15, 3))
        for j in range(4):
            k, gk = kp_brute.kp_with_grad(x - c2, np.tile(src[j] - c1, (15, 1)),
                                          np.tile(c2 - c1, (15, 1)), p)
            ref += q[j] * k
            gref += q[j] * gk
        assert rel(phi, ref) < 1e-13
        assert rel(grad, gref) < 1e-12


def test_l2l_is_exact_recentring():
    rng = np.random.default_rng(7)
    src = rng.uniform(-0.5, 0.5, (3, 3))
    q = rng.normal(size=3)
    c1, c2 = np.zeros(3), np.array([3.0, 0.0, -2.0])
    c3 = c2 + np.array([0.25, -0.25, 0.25])
    x = c3 + rng.uniform(-0.25, 0.25, (12, 3))
    for p in (2, 7, 12):
        a, ga = oracle.chain(oracle.CHAIN_M2L_L2P, p, src, q, x, c1, c2)
        b, gb = oracle.chain(oracle.CHAIN_M2L_L2L_L2P, p, src, q, x, c1, c2, c3)
        assert rel(b, a) < 1e-13
        assert rel(gb, ga) < 1e-12


def test_l2p_gradient_matches_finite_differences():
    rng = np.random.default_rng(8)
    src = rng.uniform(-0.5, 0.5, (5, 3))
    q = rng.normal(size=5)
    c1, c2 = np.zeros(3), np.array([-2.0, 2.0, 3.0])
    x = c2 + rng.uniform(-0.4, 0.4, (10, 3))
    phi, grad = oracle.chain(oracle.CHAIN_M2L_L2P, 6, src, q, x, c1, c2)
    h = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        fp, _ = oracle.chain(oracle.CHAIN_M2L_L2P, 6, src, q, x + e, c1, c2)
        fm, _ = oracle.chain(oracle.CHAIN_M2L_L2P, 6, src, q, x - e, c1, c2)
        fd = (fp - fm) / (2 * h)
        assert np.max(np.abs(fd - grad[:, a])) < 1e-8 * np.max(np.abs(grad))


# ---------------------------------------------------------- special cases
@pytest.mark.parametrize("depth", [0, 1])
def test_depth_at_most_one_is_the_direct_sum(depth):
    pos, q = W.uniform_pm1(500, 21)
    phi_d, f_d, e_d = oracle.direct(pos, q)
    phi, f, e = oracle.fmm(pos, q, depth, 6)
    assert rel(phi, phi_d) < 1e-14
    assert rel(f, f_d) < 1e-14
    assert abs(e - e_d) <= 1e-14 * abs(e_d)


def test_two_neighbouring_charges_exact():
    pos = np.array([[0.1, 0.2, 0.3], [0.35, 0.1, 0.45]])
    q = np.array([1.5, -2.0])
    r = np.linalg.norm(pos[0] - pos[1])
    _, f, e = oracle.fmm(pos, q, 2, 4)
    assert e == pytest.approx(q[0] * q[1] / r, rel=1e-15)
    # F_0 = q0 q1 (x0 - x1) / r^3 ; Newton's third law exactly
    assert np.allclose(f[0], q[0] * q[1] * (pos[0] - pos[1]) / r**3, rtol=1e-14, atol=0)
    assert np.allclose(f[0], -f[1], rtol=1e-14, atol=0)


def test_two_well_separated_charges_use_truncated_kernel():
    # level-2 boxes (0,0,0) and (2,3,0): parents adjacent, boxes not adjacent
    pos = np.array([[0.05, 0.2, 0.1], [0.6, 0.85, 0.15]])
    q = np.array([1.0, 1.0])
    for p in (1, 3, 6):
        _, _, e = oracle.fmm(pos, q, 2, p)
        ct, cs = np.array([0.125, 0.125, 0.125]), np.array([0.625, 0.875, 0.125])
        k = kp_brute.kp((pos[0] - ct)[None], (pos[1] - cs)[None], (ct - cs)[None], p)[0]
        k2 = kp_brute.kp((pos[1] - cs)[None], (pos[0] - ct)[None], (cs - ct)[None], p)[0]
        assert e == pytest.approx(0.5 * (k + k2), rel=1e-13)
        # full truncation makes the kernel symmetric
        assert k == pytest.approx(k2, rel=1e-13)


def test_energy_is_half_sum_q_phi():
    pos, q = W.uniform_gauss(3000, 31)
    phi, _, e = oracle.fmm(pos, q, 3, 5)
    assert abs(e - 0.5 * math.fsum(q * phi)) <= 1e-14 * abs(e)
    phi, _, e = oracle.direct(pos, q)
    assert abs(e - 0.5 * math.fsum(q * phi)) <= 1e-14 * abs(e)
    # and the pair form sum_{i<j} q_i q_j / r_ij
    d = np.linalg.norm(pos[:, None, :] - pos[None, :, :], axis=2)
    iu = np.triu_indices(len(q), 1)
    assert abs(e - math.fsum((q[:, None] * q[None, :] / np.where(d > 0, d, 1))[iu])) <= 1e-12 * abs(e)


def test_newton_third_law():
    pos, q = W.uniform_pm1(4096, 41)
    _, f_d, _ = oracle.direct(pos, q)
    rms = np.sqrt((f_d**2).sum(axis=1).mean())
    assert np.linalg.norm(f_d.sum(axis=0)) / (math.sqrt(len(q)) * rms) < 1e-13
    _, f, _ = oracle.fmm(pos, q, 3, 6)
    err = rel(f, f_d)
    assert np.linalg.norm(f.sum(axis=0)) / (math.sqrt(len(q)) * rms) <= 10 * err


def test_p_convergence_against_direct_sum():
    pos, q = W.uniform_pm1(2048, 51)
    phi_d, f_d, e_d = oracle.direct(pos, q)
    errs = []
    for p in (2, 4, 6, 8, 10, 12):
        phi, f, e = oracle.fmm(pos, q, 3, p)
        errs.append(rel(f, f_d))
    # roughly geometric decrease, at least 2x per two orders, ending below 1e-5
    assert all(errs[i + 1] < 0.5 * errs[i] for i in range(len(errs) - 1)), errs
    assert errs[-1] < 1e-5


def test_invariances():
    pos, q = W.uniform_gauss(1500, 61)
    phi, f, e = oracle.fmm(pos, q, 3, 5)
    # permutation of the inputs
    perm = np.random.default_rng(0).permutation(len(q))
    phi2, f2, e2 = oracle.fmm(pos[perm], q[perm], 3, 5)
    assert np.max(np.abs(phi2 - phi[perm])) <= 1e-14 * np.max(np.abs(phi))
    assert abs(e2 - e) <= 1e-14 * abs(e)
    # scaling positions and cube by 2^k: phi/l, F/l^2, E/l (exact in binary)
    lam = 4.0
    phi3, f3, e3 = oracle.fmm(pos * lam, q, 3, 5, lo=(0, 0, 0), side=lam)
    assert np.max(np.abs(phi3 - phi / lam)) <= 1e-14 * np.max(np.abs(phi / lam))
    assert np.max(np.abs(f3 - f / lam**2)) <= 1e-14 * np.max(np.abs(f / lam**2))
    assert abs(e3 - e / lam) <= 1e-14 * abs(e / lam)
    # q -> -q: phi flips, F and E unchanged
    phi4, f4, e4 = oracle.fmm(pos, -q, 3, 5)
    assert np.array_equal(phi4, -phi) and np.array_equal(f4, f) and e4 == e
    # linearity in the charges
    q2 = np.random.default_rng(1).normal(size=len(q))
    pa, _, _ = oracle.fmm(pos, q2, 3, 5)
    pb, _, _ = oracle.fmm(pos, 2.0 * q - 3.0 * q2, 3, 5)
    assert rel(pb, 2.0 * phi - 3.0 * pa) < 1e-13


def test_forces_match_finite_differences_of_energy():
    pos, q = W.uniform_gauss(300, 71)
    _, f, _ = oracle.direct(pos, q)
    h = 2e-6
    rng = np.random.default_rng(2)
    for i in rng.choice(len(q), 6, replace=False):
        for a in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, a] += h
            pm[i, a] -= h
            ep = oracle.direct(pp, q)[2]
            em = oracle.direct(pm, q)[2]
            fd = -(ep - em) / (2 * h)
            assert abs(fd - f[i, a]) <= 1e-6 * max(1.0, abs(f[i, a]))


def test_direct_sum_three_charges_closed_form():
    # equilateral triangle of side s: phi_i = (sum of the other two q) / s
    s = 0.3
    pos = np.array([[0, 0, 0], [s, 0, 0], [s / 2, s * math.sqrt(3) / 2, 0]])
    q = np.array([1.0, -2.0, 0.5])
    phi, f, e = oracle.direct(pos, q)
    assert np.allclose(phi, [(q.sum() - qi) / s for qi in q], rtol=1e-15)
    assert e == pytest.approx((q[0] * q[1] + q[0] * q[2] + q[1] * q[2]) / s, rel=1e-15)


# ------------------------------------------------------------------- tree
def test_leaf_cells_faces_and_clamping():
    L = 3
    pos = np.array([[0.0, 0.0, 0.0], [0.125, 0.25, 0.5], [1.0, 1.0, 1.0],
                    [0.124999999, 0.99999999, 0.5]])
    cells, lo, side = oracle.leaf_cells(pos, L)
    assert cells.tolist() == [[0, 0, 0], [1, 2, 4], [7, 7, 7], [0, 7, 4]]
    assert side == 1.0 and lo.tolist() == [0, 0, 0]


def test_derived_cube_rule():
    pos = np.array([[1.0, 2.0, 3.0], [1.5, 2.25, 3.1], [1.2, 2.1, 3.05]])
    _, lo, side = oracle.leaf_cells(pos, 2, side=0.0)
    assert lo.tolist() == [1.0, 2.0, 3.0] and side == 0.5
    _, lo, side = oracle.leaf_cells(pos[:1], 2, side=0.0)
    assert side == 1.0


def test_error_codes():
    pos = np.array([[0.1, 0.2, 0.3], [0.5, 0.5, 1.5]])
    with pytest.raises(oracle.OracleError) as ei:
        oracle.fmm(pos, [1.0, -1.0], 2, 3)
    assert ei.value.code == 3
    pos = np.array([[0.1, 0.2, np.nan], [0.5, 0.5, 0.5]])
    with pytest.raises(oracle.OracleError) as ei:
        oracle.fmm(pos, [1.0, -1.0], 2, 3)
    assert ei.value.code == 4
    pos = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3]])
    with pytest.raises(oracle.OracleError) as ei:
        oracle.fmm(pos, [1.0, -1.0], 2, 3)
    assert ei.value.code == 5


def test_sampled_targets_equal_full_run():
    pos, q = W.uniform_gauss(5000, 81)
    phi, f, _ = oracle.fmm(pos, q, 4, 4)
    t = np.random.default_rng(3).choice(len(q), 50, replace=False)
    phs, fs, es = oracle.fmm(pos, q, 4, 4, targets=t)
    assert es is None
    assert np.array_equal(phs, phi[t]) and np.array_equal(fs, f[t])
    phd, fd, _ = oracle.direct(pos, q)
    phs, fs, _ = oracle.direct(pos, q, targets=t)
    assert np.array_equal(phs, phd[t]) and np.array_equal(fs, fd[t])
