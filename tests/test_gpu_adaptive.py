"""GPU parity of the adaptive-octree FMM (leaf_max > 0) through the C ABI.

* FP64 GPU against the oracle's adaptive FMM on the same tree: phi, F and E
  to rounding (1e-12), and the tree's integer statistics (boxes, leaves,
  deepest level, U / V / W / X list sizes, P2P and M2L pair counts) exactly.
* Mixed precision against the same oracle: relative E <= 1e-6 and RMS F
  <= 1e-5, for every M2L form.
* Special cases: a tree that is the uniform one (equals the uniform GPU path),
  the root as the only leaf (direct sum), the depth cap, coincident points,
  empty boxes, determinism and the adjoint (dE/dq = phi, dE/dx = -F).
* The clustered workload at full size (10^6 three-site clusters, leaves of at
  most 64 sites, p = 10): tree statistics exactly equal to the oracle's; FP64
  GPU at p = 2 against the oracle at p = 2 on every particle; mixed p = 10
  against FP64 p = 10 (energy gate) and against the direct sum on sampled
  particles (truncation bound).
"""
import numpy as np
import pytest

import oracle
from gpu_util import assert_close, B, log, rel, run_gpu
from paper_2209_13121_amd import workloads as W

pytestmark = pytest.mark.gpu

MIXED = B.FMM_PREC_MIXED
FP64 = B.FMM_PREC_FP64


def clustered(n, seed, frac=0.5, width=0.04, centre=0.3):
    rng = np.random.default_rng(seed)
    m = int(n * frac)
    pos = np.concatenate([rng.random((n - m, 3)),
                          np.clip(centre + width * rng.standard_normal((m, 3)), 0.0, 1.0)])
    q = rng.standard_normal(n)
    q -= q.mean()
    return pos, q


CASES = {
    # name: (inputs, leaf_max, depth cap, p)
    "blob-n3000-leaf16-p6": (lambda: clustered(3000, 21), 16, 6, 6),
    "blob-n5000-leaf8-p4": (lambda: clustered(5000, 22, frac=0.7, width=0.02), 8, 7, 4),
    "clusters-n3000-leaf24-p8": (lambda: W.molecular_clusters(1000, 23)[:2], 24, 7, 8),
    # the order of the cluster workload (p = 10): its own operator staging
    "clusters-n3000-leaf24-p10": (lambda: W.molecular_clusters(1000, 23)[:2], 24, 7, 10),
}


def _oracle(name):
    make, leaf_max, cap, p = CASES[name]
    pos, q = make()
    side = 0.0 if name.startswith("clusters") else 1.0
    phi, force, e, st = oracle.fmm_adaptive(pos, q, leaf_max, cap, p, side=side)
    return pos, q, side, (phi, force, e, st)


@pytest.mark.parametrize("name", sorted(CASES))
def test_fp64_matches_oracle(name):
    make, leaf_max, cap, p = CASES[name]
    pos, q, side, (phi_o, f_o, e_o, st_o) = _oracle(name)
    log(f"[adaptive fp64] {name}: oracle tree {st_o}")
    st_g = {}
    phi, force, e, st = run_gpu(pos, q, cap, p, FP64, side=side, leaf_max=leaf_max, stats=st_g)
    assert st_g == st_o
    assert st_o["w"] > 0 and st_o["x"] > 0
    assert_close(phi, phi_o, 1e-12, what="phi")
    assert_close(force, f_o, 1e-12, what="force")
    assert abs(e - e_o) <= 1e-12 * abs(e_o)


@pytest.mark.parametrize("kind", ["auto", "f32", "bf16x3", "f16x2"])
@pytest.mark.parametrize("name", sorted(CASES))
def test_mixed_within_gate(name, kind):
    make, leaf_max, cap, p = CASES[name]
    pos, q, side, (phi_o, f_o, e_o, _) = _oracle(name)
    mk = getattr(B, "FMM_M2L_" + kind.upper())
    log(f"[adaptive mixed] {name} {kind}")
    phi, force, e, st = run_gpu(pos, q, cap, p, MIXED, side=side, leaf_max=leaf_max, m2l_kind=mk)
    assert abs(e - e_o) / abs(e_o) <= 1e-6
    assert_close(force, f_o, 1e-5, what="force")
    assert_close(phi, phi_o, 1e-5, what="phi")


def test_uniform_tree_equals_uniform_path():
    # leaf_max = 1 with enough particles divides every box down to the cap.
    pos, q = W.uniform_gauss(20000, 24)
    st = {}
    phi_a, f_a, e_a, _ = run_gpu(pos, q, 3, 6, FP64, leaf_max=1, stats=st)
    assert st["leaves"] == 512 and st["w"] == 0 and st["x"] == 0
    phi_u, f_u, e_u, _ = run_gpu(pos, q, 3, 6, FP64)
    assert_close(phi_a, phi_u, 1e-13, what="phi_a")
    assert_close(f_a, f_u, 1e-13, what="f_a")
    assert abs(e_a - e_u) <= 1e-13 * abs(e_u)


def test_root_leaf_is_direct_sum():
    pos, q = clustered(200, 25)
    st = {}
    for prec, tol in ((FP64, 1e-13), (MIXED, 1e-5)):
        phi, force, e, _ = run_gpu(pos, q, 6, 6, prec, leaf_max=500, stats=st)
        assert st["boxes"] == 1 and st["leaves"] == 1
        phi_d, f_d, e_d = oracle.direct(pos, q)
        assert rel(phi, phi_d) < tol
        assert rel(force, f_d) < tol


def test_depth_cap_and_empty_boxes():
    rng = np.random.default_rng(26)
    pos = np.concatenate([0.02 + 0.3 * rng.random((150, 3)), 0.61 + 1e-4 * rng.random((100, 3))])
    q = rng.standard_normal(250)
    phi_o, f_o, e_o, st_o = oracle.fmm_adaptive(pos, q, 4, 4, 5)
    st = {}
    phi, force, e, _ = run_gpu(pos, q, 4, 5, FP64, leaf_max=4, stats=st)
    assert st == st_o and st["deepest"] == 4
    assert_close(phi, phi_o, 1e-12, what="phi")
    assert_close(force, f_o, 1e-12, what="force")


def test_coincident_points_flagged():
    pos, q = clustered(400, 27)
    pos[7] = pos[300]
    with pytest.raises(B.FMMError) as ei:
        run_gpu(pos, q, 6, 4, FP64, leaf_max=8)
    assert ei.value.status == 5  # FMM_E_COINCIDENT


def test_deterministic():
    pos, q = clustered(4000, 28)
    for prec in (FP64, MIXED):
        a = run_gpu(pos, q, 6, 6, prec, leaf_max=16)
        b = run_gpu(pos, q, 6, 6, prec, leaf_max=16)
        assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_adjoint_on_adaptive_tree():
    import torch
    pos, q = clustered(3000, 29)
    dev = torch.device("cuda:0")
    tp = torch.from_numpy(pos).to(dev)
    tq = torch.from_numpy(q).to(dev)
    f = B.FMM(tp, p=6, depth=6, leaf_max=16)
    phi, force, energy = f.evaluate(tq)
    g = torch.tensor([0.5], dtype=torch.float64, device=dev)
    dx = torch.empty((len(q), 3), dtype=torch.float64, device=dev)
    dq = torch.empty(len(q), dtype=torch.float64, device=dev)
    B.fmm_backward(f.plan, g, dx, dq)
    torch.cuda.synchronize()
    assert torch.equal(dq, 0.5 * phi)
    assert torch.equal(dx, -0.5 * force)
    f.close()


@pytest.mark.parametrize("leaf_max,depth", [(0, 4), (0, 5), (64, 7)])
def test_mixed_potential_has_no_drift_on_neutral_clusters(leaf_max, depth):
    # Neutral three-site clusters: the leaf multipoles are summed in FP64, so
    # the mixed potential carries no coherent, density-shaped offset (an FP32
    # sum gave 3e-4 of phi at depth 4 on this input); energy and forces are
    # insensitive to a constant offset, phi is not.
    pos, q, _ = W.molecular_clusters(100_000, 32)
    a = run_gpu(pos, q, depth, 6, FP64, side=0.0, leaf_max=leaf_max)
    b = run_gpu(pos, q, depth, 6, MIXED, side=0.0, leaf_max=leaf_max)
    d = b[0] - a[0]
    log(f"[drift] leaf_max {leaf_max} depth {depth}: phi rel {rel(b[0], a[0]):.3g} mean {d.mean():.3g}")
    assert_close(b[0], a[0], 1e-5, what="b")
    assert abs(d.mean()) < 1e-5 * np.sqrt(np.mean(a[0] ** 2))


@pytest.fixture(scope="module")
def clusters_full():
    wl = W.CLUSTERS
    pos, q = wl.make()
    return wl, pos, q


def test_clusters_full_size_tree_and_low_order_parity(clusters_full):
    wl, pos, q = clusters_full
    log(f"[adaptive full] {wl.name}: oracle p=2")
    phi_o, f_o, e_o, st_o = oracle.fmm_adaptive(pos, q, wl.leaf_max, wl.max_depth, 2, side=0.0)
    st = {}
    phi, force, e, _ = run_gpu(pos, q, wl.max_depth, 2, FP64, side=0.0, leaf_max=wl.leaf_max,
                               stats=st)
    log(f"[adaptive full] tree {st}")
    assert st == st_o
    assert_close(phi, phi_o, 1e-12, what="phi")
    assert_close(force, f_o, 1e-12, what="force")
    assert abs(e - e_o) <= 1e-12 * abs(e_o)


def test_clusters_full_size_mixed(clusters_full):
    wl, pos, q = clusters_full
    log(f"[adaptive full] {wl.name}: fp64 and mixed at p={wl.p}")
    phi64, f64, e64, _ = run_gpu(pos, q, wl.max_depth, wl.p, FP64, side=0.0, leaf_max=wl.leaf_max)
    phim, fm, em, _ = run_gpu(pos, q, wl.max_depth, wl.p, MIXED, side=0.0, leaf_max=wl.leaf_max)
    assert abs(em - e64) / abs(e64) <= 1e-6
    assert_close(fm, f64, 1e-5, what="fm")
    # both against the exact sum on sampled particles: the truncation error of
    # p = 10 on this tree is about 1e-6 (oracle, smaller sizes); the
    # per-particle bound is a truncation bound (a pair's K_p error reaches 2e-4
    # at p = 10), loose next to the oracle-parity ones but far below the O(1)
    # error of a wrong box
    rng = np.random.default_rng(30)
    idx = rng.choice(len(q), 256, replace=False)
    phi_d, f_d, _ = oracle.direct(pos, q, targets=idx)
    assert_close(phi64[idx], phi_d, 2e-5, elem_tol=1e-2, what="phi64 vs direct")
    assert_close(phim[idx], phi_d, 2e-5, elem_tol=1e-2, what="phim vs direct")
    assert_close(f64[idx], f_d, 1e-4, elem_tol=1e-2, what="f64 vs direct")


# 10^5 clusters (3e5 sites), leaves of at most 64, p = 10: about 200 M2L
# work-groups, so every XCD runs whole groups besides the split tail parts
# (the small cases above have fewer than 128 groups, all of them split).
MEDIUM = (100_000, 33, 64, 7, 10)


@pytest.fixture(scope="module")
def medium_clusters():
    nc, seed, leaf_max, cap, p = MEDIUM
    pos, q, _ = W.molecular_clusters(nc, seed)
    log(f"[adaptive medium] oracle p={p} on {len(q)} sites")
    ref = oracle.fmm_adaptive(pos, q, leaf_max, cap, p, side=0.0)
    return pos, q, ref


def test_medium_clusters_fp64(medium_clusters):
    pos, q, (phi_o, f_o, e_o, st_o) = medium_clusters
    _, _, leaf_max, cap, p = MEDIUM
    st = {}
    phi, force, e, _ = run_gpu(pos, q, cap, p, FP64, side=0.0, leaf_max=leaf_max, stats=st)
    assert st == st_o
    assert_close(phi, phi_o, 1e-12, what="phi")
    assert_close(force, f_o, 1e-12, what="force")
    assert abs(e - e_o) <= 1e-12 * abs(e_o)


@pytest.mark.parametrize("kind", ["auto", "f32", "bf16x3", "f16x2"])
def test_medium_clusters_mixed(medium_clusters, kind):
    pos, q, (phi_o, f_o, e_o, _) = medium_clusters
    _, _, leaf_max, cap, p = MEDIUM
    mk = getattr(B, "FMM_M2L_" + kind.upper())
    log(f"[adaptive medium mixed] {kind}")
    phi, force, e, _ = run_gpu(pos, q, cap, p, MIXED, side=0.0, leaf_max=leaf_max, m2l_kind=mk)
    log(f"  dE {abs(e - e_o) / abs(e_o):.2e}")
    assert abs(e - e_o) / abs(e_o) <= 1e-6
    assert_close(force, f_o, 1e-5, what="force")
    assert_close(phi, phi_o, 1e-5, what="phi")
