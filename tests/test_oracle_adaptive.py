"""Pins of the oracle's adaptive-octree FMM (CPU only).

The adaptive oracle (U, V, W, X lists; Cheng, Greengard & Rokhlin 1999,
sec. 4) is checked against things it does not share code with:
  * a pair-by-pair brute force of the adaptive method's result from its
    definition (tests/kp_brute.py: every pair is handled by exactly one of
    M2L at the first separated level, M2P, P2L or the exact 1/r, each a
    truncated Taylor kernel evaluated without spherical harmonics);
  * the uniform-tree oracle, on inputs whose adaptive tree is uniform;
  * the direct sum, when the root is the only box, and in the limit of p;
  * list duality (b is in W(c) exactly when c is in X(b));
  * planted mistakes in a copy of the adaptive code, each rejected.
"""
import os
import subprocess

import numpy as np
import pytest

import kp_brute
import oracle
from oracle import build as obuild
from paper_2209_13121_amd import workloads as W


def clustered(n, seed, frac=0.5, width=0.04, centre=0.3):
    """Half uniform in the unit cube, half a tight Gaussian blob: trees with
    leaves on several levels, so W and X are not empty."""
    rng = np.random.default_rng(seed)
    m = int(n * frac)
    pos = np.concatenate([rng.random((n - m, 3)),
                          np.clip(centre + width * rng.standard_normal((m, 3)), 0.0, 1.0)])
    q = rng.standard_normal(n)
    q -= q.mean()
    return pos, q


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("n,seed,leaf_max,max_depth,p", [
    (300, 5, 6, 5, 3),
    (240, 6, 10, 4, 4),
    (200, 7, 3, 6, 2),
])
def test_adaptive_matches_pairwise_brute_force(n, seed, leaf_max, max_depth, p):
    pos, q = clustered(n, seed)
    phi, force, energy, st = oracle.fmm_adaptive(pos, q, leaf_max, max_depth, p)
    phi_b, grad_b, counts = kp_brute.fmm_adaptive_brute(pos, q, leaf_max, max_depth, p)
    assert counts["m2p"] > 0 and counts["p2l"] > 0 and counts["m2l"] > 0
    assert rel(phi, phi_b) < 1e-12
    assert rel(force, -q[:, None] * grad_b) < 1e-12
    assert st["p2p_pairs"] == counts["p2p"]
    assert abs(energy - 0.5 * np.dot(q, phi)) <= 1e-13 * np.abs(q * phi).sum()


def test_adaptive_list_duality():
    pos, q = clustered(400, 8)
    _, _, _, st = oracle.fmm_adaptive(pos, q, 5, 6, 2)
    assert st["w"] == st["x"] > 0
    assert st["deepest"] >= 4


@pytest.mark.parametrize("depth", [2, 3])
def test_uniform_tree_equals_uniform_fmm(depth):
    # With leaf_max = 1 and enough particles every box above max_depth holds
    # more than one particle, so the adaptive tree is the uniform one.
    pos, q = W.uniform_gauss(3000, 11)
    phi, force, e, st = oracle.fmm_adaptive(pos, q, 1, depth, 4)
    assert st["leaves"] == 8 ** depth and st["w"] == 0 and st["x"] == 0
    phi_u, force_u, e_u = oracle.fmm(pos, q, depth, 4)
    assert rel(phi, phi_u) < 1e-13
    assert rel(force, force_u) < 1e-13
    assert abs(e - e_u) <= 1e-13 * abs(e_u)


def test_root_leaf_is_direct_sum():
    pos, q = clustered(150, 12)
    phi, force, e, st = oracle.fmm_adaptive(pos, q, 200, 6, 6)
    assert st["boxes"] == 1 and st["leaves"] == 1
    phi_d, force_d, e_d = oracle.direct(pos, q)
    assert rel(phi, phi_d) < 1e-14
    assert rel(force, force_d) < 1e-14


def test_depth_cap_holds():
    # 60 points in a region far smaller than the finest box: the cap stops
    # the division, and the result still matches the brute force.
    rng = np.random.default_rng(13)
    pos = np.concatenate([rng.random((60, 3)), 0.61 + 1e-4 * rng.random((60, 3))])
    q = rng.standard_normal(120)
    phi, force, e, st = oracle.fmm_adaptive(pos, q, 4, 3, 3)
    assert st["deepest"] == 3
    phi_b, grad_b, _ = kp_brute.fmm_adaptive_brute(pos, q, 4, 3, 3)
    assert rel(phi, phi_b) < 1e-12
    assert rel(force, -q[:, None] * grad_b) < 1e-12


def test_adaptive_p_convergence():
    pos, q = clustered(2000, 14)
    phi_d, force_d, _ = oracle.direct(pos, q)
    errs = [rel(oracle.fmm_adaptive(pos, q, 16, 8, p)[0], phi_d) for p in (2, 4, 6, 8, 10)]
    # geometric decrease, roughly a factor 5-10 per two orders here
    assert all(b < 0.3 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-5


def test_adaptive_derived_cube_and_scaling():
    # Scaling positions by 2^k (derived cube) scales phi by 2^-k exactly.
    pos, q = clustered(300, 15)
    phi, force, e, _ = oracle.fmm_adaptive(pos, q, 8, 6, 4, side=0.0)
    phi2, force2, e2, _ = oracle.fmm_adaptive(pos * 8.0, q, 8, 6, 4, side=0.0)
    assert np.array_equal(phi2 * 8.0, phi)
    assert np.array_equal(force2 * 64.0, force)


ADAPTIVE_MUTATIONS = {
    # P2L without the conjugate
    "p2l_conj": ("for (int i = 0; i < nharm(p); ++i) L[i] += q * conj(Ih[i]);",
                 "for (int i = 0; i < nharm(p); ++i) L[i] += q * Ih[i];"),
    # M2P gradient x component with the order shift reversed
    "m2p_grad": ("grad[0] = creal(0.5 * (Lk[hidx(1, -1)] - Lk[hidx(1, 1)]));",
                 "grad[0] = creal(0.5 * (Lk[hidx(1, 1)] - Lk[hidx(1, -1)]));"),
    # W also takes same-level boxes (already in V)
    "w_level": ("if (C->level > B->level) alist_add(W, c);",
                "if (C->level >= B->level) alist_add(W, c);"),
    # X keeps coarse leaves adjacent to the box (already in U)
    "x_adjacent": ("if (!aadjacent(B, C)) alist_add(X, c);", "alist_add(X, c);"),
    # V keeps children of the parent's colleagues that touch the box
    "v_adjacent": ("if (!aadjacent(B, T->box + T->box[col].child0 + ch)) alist_add(V, T->box[col].child0 + ch);",
                   "alist_add(V, T->box[col].child0 + ch);"),
    # adjacency of open cubes (boxes that only share a face count as separated)
    "adj_open": ("if (alo > bhi || blo > ahi) return 0;", "if (alo >= bhi || blo >= ahi) return 0;"),
    # the parent's local expansion not passed down at level 3
    "l2l_level": ("if (l >= 3) {\n        double cp[3];", "if (l >= 4) {\n        double cp[3];"),
}


@pytest.fixture(scope="module")
def adaptive_reference():
    pos, q = clustered(180, 16)
    phi_b, grad_b, _ = kp_brute.fmm_adaptive_brute(pos, q, 5, 5, 3)
    return pos, q, phi_b, grad_b


def _build_variant(tmp_path, name, old, new):
    src = open(obuild.SRC).read()
    assert src.count(old) == 1, f"mutation {name} does not match the oracle source"
    path = os.path.join(tmp_path, f"oracle_{name}.c")
    with open(path, "w") as f:
        f.write(src.replace(old, new))
    lib = os.path.join(tmp_path, f"liboracle_{name}.so")
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-fcx-limited-range", path, "-o", lib, "-lm"], check=True)
    return oracle.load_library(lib)


@pytest.mark.parametrize("name", sorted(ADAPTIVE_MUTATIONS))
def test_adaptive_planted_mistake_is_caught(tmp_path, adaptive_reference, name):
    pos, q, phi_b, grad_b = adaptive_reference
    old, new = ADAPTIVE_MUTATIONS[name]
    lib = _build_variant(str(tmp_path), name, old, new)
    phi, f, _, _ = oracle.fmm_adaptive(pos, q, 5, 5, 3, lib=lib)
    grad = -f / q[:, None]
    assert max(rel(phi, phi_b), rel(grad, grad_b)) > 1e-6, name


def test_molecular_clusters_geometry():
    pos, q, side = W.molecular_clusters(500, 3)
    s = pos.reshape(-1, 3, 3)
    b1 = np.linalg.norm(s[:, 1] - s[:, 0], axis=1)
    b2 = np.linalg.norm(s[:, 2] - s[:, 0], axis=1)
    assert np.allclose(b1, W.CLUSTER_BOND_NM, rtol=1e-12) and np.allclose(b2, W.CLUSTER_BOND_NM, rtol=1e-12)
    cosang = ((s[:, 1] - s[:, 0]) * (s[:, 2] - s[:, 0])).sum(1) / (b1 * b2)
    assert np.allclose(np.degrees(np.arccos(cosang)), W.CLUSTER_ANGLE_DEG, atol=1e-9)
    assert np.allclose(q.reshape(-1, 3).sum(1), 0.0, atol=1e-15)
    assert len(q) == 1500 and np.all(s[:, 0] >= 0) and np.all(s[:, 0] <= side)
    # denser near the blob centres: the first sites are not uniform
    counts = np.histogramdd(s[:, 0], bins=4, range=[(0, side)] * 3)[0]
    assert counts.max() > 2.0 * counts.mean()
