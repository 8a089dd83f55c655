"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Tolerances
  * FP64 mode: normwise relative error of phi and F, and relative error of E,
    <= 1e-12 against the oracle FMM with the same cube, depth and p.  Both
    sides evaluate the same truncated expansion in FP64 in different bases and
    summation orders, so only rounding separates them.
  * Mixed mode: relative E <= 1e-6, normwise relative RMS force <= 1e-5 and
    potential <= 1e-5 against the FP64 oracle FMM.
  * Integer work (leaf cells, the resolved cube): bit-exact.
"""
import json
import os

import numpy as np
import pytest

import oracle
from gpu_util import assert_close, B, half_sum_q_phi, log, rel, run_gpu, energy_rel
from paper_2209_13121_amd import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))

# (name, n, charges, seed, depth, p)
FP64_CASES = [
    ("small-workload", W.SMALL.n, W.SMALL.charges, W.SMALL.seed, W.SMALL.depth, W.SMALL.p),
    ("n2000-L2-p6", 2000, "gauss", 11, 2, 6),
    ("n5000-L4-p5-empty-leaves", 5000, "gauss", 12, 4, 5),
    ("n3000-L3-p8", 3000, "pm1", 13, 3, 8),
    ("n1500-L3-p0", 1500, "gauss", 14, 3, 0),
    ("n1500-L3-p1", 1500, "gauss", 15, 3, 1),
    ("n1000-L3-p12", 1000, "gauss", 16, 3, 12),
    ("n777-L1-direct", 777, "gauss", 17, 1, 3),
    ("n513-L0-direct", 513, "pm1", 18, 0, 2),
    ("n20011-L4-p6-ragged", 20011, "gauss", 19, 4, 6),
]


def make(n, charges, seed):
    gen = W.uniform_pm1 if charges == "pm1" else W.uniform_gauss
    return gen(n, seed)


@pytest.mark.parametrize("case", FP64_CASES, ids=[c[0] for c in FP64_CASES])
def test_fp64_matches_oracle(case):
    name, n, charges, seed, depth, p = case
    log(f"[fp64] {name}")
    pos, q = make(n, charges, seed)
    phi, force, e, _ = run_gpu(pos, q, depth, p)
    phi_o, force_o, e_o = oracle.fmm(pos, q, depth, p)
    assert_close(phi, phi_o, 1e-12, what="phi")
    assert_close(force, force_o, 1e-12, what="force")
    assert energy_rel(e, e_o) <= 1e-12
    assert energy_rel(e, half_sum_q_phi(q, phi)) <= 1e-13


def test_fp64_nonunit_and_derived_cube():
    log("[fp64] non-unit cube")
    pos, q = W.uniform_gauss(3000, 21)
    lo, side = np.array([-3.0, 1.5, 0.25]), 2.5
    pos = lo + pos * side * 0.999
    phi, force, e, _ = run_gpu(pos, q, 3, 6, lo=lo, side=side)
    phi_o, force_o, e_o = oracle.fmm(pos, q, 3, 6, lo=lo, side=side)
    assert_close(phi, phi_o, 1e-12, what="phi")
    assert_close(force, force_o, 1e-12, what="force")
    assert energy_rel(e, e_o) <= 1e-12
    log("[fp64] derived cube")
    phi, force, e, _ = run_gpu(pos, q, 3, 6, side=0.0)
    phi_o, force_o, e_o = oracle.fmm(pos, q, 3, 6, side=0.0)
    assert_close(phi, phi_o, 1e-12, what="phi")
    assert_close(force, force_o, 1e-12, what="force")
    assert energy_rel(e, e_o) <= 1e-12


@pytest.mark.parametrize("depth,side", [(3, 1.0), (5, 1.0), (4, 0.0)])
def test_leaf_cells_and_cube_bit_exact(depth, side):
    import torch
    log(f"[tree] depth {depth} side {side}")
    pos, _ = W.uniform_gauss(10000, 31 + depth)
    # points exactly on internal faces and on the top face
    pos[:8] = np.array([[0.5, 0.25, 0.125], [1.0, 1.0, 1.0], [0.0, 0.0, 0.0],
                        [0.75, 0.999999999999, 0.5], [0.125, 0.375, 0.625],
                        [1 / 3, 2 / 3, 0.1], [0.3125, 0.6875, 0.0625], [0.5, 0.5, 0.5]])
    dev = torch.device("cuda:0")
    tp = torch.from_numpy(pos).to(dev)
    f = B.FMM(tp, p=2, depth=depth, side=side)
    cells = torch.empty((len(pos), 3), dtype=torch.int32, device=dev)
    leaf = torch.empty(len(pos), dtype=torch.int32, device=dev)
    B.fmm_plan_leaves(f.plan, cells, leaf)
    lo_g, side_g = B.fmm_plan_cube(f.plan)
    assert f.check() == 0
    cells_o, lo_o, side_o = oracle.leaf_cells(pos, depth, side=side)
    assert np.array_equal(cells.cpu().numpy(), cells_o)
    assert lo_g == list(lo_o) and side_g == side_o
    # The device's leaf slots are checked against properties of an
    # octree-consistent Hilbert order, not against a host copy of the curve:
    # a bijection between occupied cells and slots in [0, 8^depth); at every
    # coarser level the slot prefix is a bijection of the ancestor cell; and
    # consecutive slots are face-adjacent cells.
    lv = leaf.cpu().numpy().astype(np.int64)
    assert lv.min() >= 0 and lv.max() < 8 ** depth
    for lvl in range(1, depth + 1):
        sh = depth - lvl
        c = cells_o.astype(np.int64) >> sh
        key = (c[:, 0] << 42) | (c[:, 1] << 21) | c[:, 2]
        pairs = np.unique(np.stack([key, lv >> (3 * sh)], axis=1), axis=0)
        assert len(np.unique(pairs[:, 0])) == len(pairs) == len(np.unique(pairs[:, 1]))
    slots, first = np.unique(lv, return_index=True)
    cs = cells_o[first].astype(np.int64)
    step = np.abs(np.diff(cs, axis=0)).sum(axis=1)
    consecutive = np.diff(slots) == 1
    assert consecutive.sum() > 0 and np.all(step[consecutive] == 1)
    if depth == 3:
        assert len(slots) == 512  # every cell occupied: the whole curve
    f.close()


def test_headline_fp64_sampled():
    """Full-size headline workload, FP64 mode, in the launch configuration the
    benchmark uses; sampled targets against the oracle one by one."""
    wl = W.HEADLINE
    log(f"[fp64] {wl.name} (sampled)")
    pos, q = wl.make()
    phi, force, e, _ = run_gpu(pos, q, wl.depth, wl.p)
    t = np.random.default_rng(5).choice(wl.n, 256, replace=False)
    phi_o, force_o, _ = oracle.fmm(pos, q, wl.depth, wl.p, targets=t)
    assert_close(phi[t], phi_o, 1e-12, what="phi")
    assert_close(force[t], force_o, 1e-12, what="force")
    assert energy_rel(e, half_sum_q_phi(q, phi)) <= 1e-12
    golden = os.path.join(HERE, "golden", "headline_oracle.json")
    if os.path.exists(golden):
        ref = json.load(open(golden))[wl.name]
        assert energy_rel(e, ref["energy"]) <= 1e-12


MIXED_CASES = [
    ("small-workload", W.SMALL.n, W.SMALL.charges, W.SMALL.seed, W.SMALL.depth, W.SMALL.p),
    ("n30000-L4-p8", 30000, "gauss", 41, 4, 8),
    ("n8000-L3-p10", 8000, "pm1", 42, 3, 10),
    ("n2000-L2-p6", 2000, "gauss", 43, 2, 6),
    ("n3000-L3-p1", 3000, "pm1", 44, 3, 1),
    ("n3000-L3-p12", 3000, "gauss", 45, 3, 12),
]


MIXED_KINDS = {"f32": B.FMM_M2L_F32, "bf16x3": B.FMM_M2L_BF16X3, "f16x2": B.FMM_M2L_F16X2,
               "auto": B.FMM_M2L_AUTO}


@pytest.mark.parametrize("kind", sorted(MIXED_KINDS))
@pytest.mark.parametrize("case", MIXED_CASES, ids=[c[0] for c in MIXED_CASES])
def test_mixed_within_gate(case, kind):
    # Three BF16 pieces reproduce FP32 operands exactly and the dropped piece
    # products are below 2^-24 relative: both M2L forms share the FP32 gate.
    name, n, charges, seed, depth, p = case
    log(f"[mixed {kind}] {name}")
    pos, q = make(n, charges, seed)
    phi, force, e, _ = run_gpu(pos, q, depth, p, precision=B.FMM_PREC_MIXED,
                               m2l_kind=MIXED_KINDS[kind])
    phi_o, force_o, e_o = oracle.fmm(pos, q, depth, p)
    log(f"  dE {energy_rel(e, e_o):.2e} dF {rel(force, force_o):.2e} dphi {rel(phi, phi_o):.2e}")
    assert energy_rel(e, e_o) <= 1e-6
    assert_close(force, force_o, 1e-5, what="force")
    assert_close(phi, phi_o, 1e-5, what="phi")
    assert energy_rel(e, half_sum_q_phi(q, phi)) <= 1e-13


@pytest.mark.parametrize("kind", ["f32", "bf16x3", "f16x2"])
def test_mixed_charge_scales(kind):
    # The FP16 form scales operands by powers of two (per operator row and
    # column, per source box), so its accuracy must not depend on the charge
    # magnitude, nor suffer where one region's charges dwarf the rest's.
    pos, q = make(20000, "gauss", 46)
    cases = [("x1e20", q * 1e20), ("x1e-20", q * 1e-20)]
    q2 = q.copy()
    q2[pos[:, 0] < 0.25] *= 1e8  # one region 1e8 times stronger
    cases.append(("region-1e8", q2))
    for name, qq in cases:
        log(f"[mixed {kind}] charge scale {name}")
        phi, force, e, _ = run_gpu(pos, qq, 4, 8, precision=B.FMM_PREC_MIXED,
                                   m2l_kind=MIXED_KINDS[kind])
        phi_o, force_o, e_o = oracle.fmm(pos, qq, 4, 8)
        log(f"  dE {energy_rel(e, e_o):.2e} dF {rel(force, force_o):.2e} dphi {rel(phi, phi_o):.2e}")
        assert energy_rel(e, e_o) <= 1e-6
        assert_close(force, force_o, 1e-5, what="force")
        assert_close(phi, phi_o, 1e-5, what="phi")


def test_mixed_bf16x2_accuracy():
    # Two pieces carry about 16 significant bits per product: a documented
    # looser mode, checked against its own bound (about 2^-16 of the far field).
    n, depth, p = 30000, 4, 8
    log("[mixed bf16x2] n30000-L4-p8")
    pos, q = make(n, "gauss", 41)
    phi, force, e, _ = run_gpu(pos, q, depth, p, precision=B.FMM_PREC_MIXED,
                               m2l_kind=B.FMM_M2L_BF16X2)
    phi_o, force_o, e_o = oracle.fmm(pos, q, depth, p)
    log(f"  dE {energy_rel(e, e_o):.2e} dF {rel(force, force_o):.2e} dphi {rel(phi, phi_o):.2e}")
    assert_close(phi, phi_o, 1e-4, what="phi")
    assert_close(force, force_o, 1e-4, what="force")
    assert energy_rel(e, e_o) <= 1e-4


@pytest.mark.parametrize("kind", ["f32", "bf16x3", "f16x2"])
def test_headline_mixed_sampled(kind):
    wl = W.HEADLINE
    log(f"[mixed {kind}] {wl.name} (sampled)")
    pos, q = wl.make()
    phi, force, e, _ = run_gpu(pos, q, wl.depth, wl.p, precision=B.FMM_PREC_MIXED,
                               m2l_kind=MIXED_KINDS[kind])
    t = np.random.default_rng(6).choice(wl.n, 512, replace=False)
    phi_o, force_o, _ = oracle.fmm(pos, q, wl.depth, wl.p, targets=t)
    log(f"  sampled dF {rel(force[t], force_o):.2e} dphi {rel(phi[t], phi_o):.2e}")
    assert_close(force[t], force_o, 1e-5, what="force")
    assert_close(phi[t], phi_o, 1e-5, what="phi")
    assert energy_rel(e, half_sum_q_phi(q, phi)) <= 1e-12
    golden = os.path.join(HERE, "golden", "headline_oracle.json")
    if os.path.exists(golden):
        ref = json.load(open(golden))[wl.name]
        log(f"  dE {energy_rel(e, ref['energy']):.2e}")
        assert energy_rel(e, ref["energy"]) <= 1e-6


@pytest.mark.parametrize("precision,kind", [(B.FMM_PREC_FP64, B.FMM_M2L_AUTO),
                                            (B.FMM_PREC_MIXED, B.FMM_M2L_F32),
                                            (B.FMM_PREC_MIXED, B.FMM_M2L_BF16X3),
                                            (B.FMM_PREC_MIXED, B.FMM_M2L_F16X2)])
def test_deterministic(precision, kind):
    log(f"[determinism] precision {precision} m2l {kind}")
    pos, q = W.uniform_gauss(50000, 51)
    a = run_gpu(pos, q, 4, 6, precision=precision, m2l_kind=kind)
    b = run_gpu(pos, q, 4, 6, precision=precision, m2l_kind=kind)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1]) and a[2] == b[2]


def test_edge_cases():
    log("[edge] n=1, n=2, one leaf, empty leaves")
    phi, force, e, _ = run_gpu(np.array([[0.3, 0.4, 0.5]]), np.array([2.0]), 3, 4)
    assert phi[0] == 0.0 and np.all(force == 0.0) and e == 0.0
    pos = np.array([[0.1, 0.1, 0.1], [0.9, 0.8, 0.85]])
    q = np.array([1.0, -2.0])
    for depth in (0, 2, 3):
        phi, force, e, _ = run_gpu(pos, q, depth, 6)
        phi_o, force_o, e_o = oracle.fmm(pos, q, depth, 6)
        assert_close(phi, phi_o, 1e-12, what="phi")
        assert energy_rel(e, e_o) <= 1e-12
    # every particle in one leaf of a deep tree: only P2P contributes
    rng = np.random.default_rng(3)
    pos = 0.2 + 0.01 * rng.random((300, 3))
    q = rng.normal(size=300)
    phi, force, e, _ = run_gpu(pos, q, 4, 5)
    phi_d, force_d, e_d = oracle.direct(pos, q)
    assert_close(phi, phi_d, 1e-13, what="phi")
    assert_close(force, force_d, 1e-13, what="force")


def test_device_error_flags():
    log("[errors] out of cube, non-finite, coincident")
    pos, q = W.uniform_gauss(1000, 61)
    bad = pos.copy()
    bad[10] = [0.5, 1.5, 0.5]
    assert run_gpu(bad, q, 3, 4, check=False)[3] == 3
    bad = pos.copy()
    bad[20, 1] = np.nan
    assert run_gpu(bad, q, 3, 4, check=False)[3] == 4
    bad = pos.copy()
    bad[30] = bad[31]
    for prec in (B.FMM_PREC_FP64, B.FMM_PREC_MIXED):
        assert run_gpu(bad, q, 3, 4, precision=prec, check=False)[3] == 5


def test_optional_outputs_and_reuse():
    import torch
    log("[api] optional outputs, plan reuse")
    pos, q = W.uniform_gauss(4000, 71)
    dev = torch.device("cuda:0")
    f = B.FMM(torch.from_numpy(pos).to(dev), p=5, depth=3)
    tq = torch.from_numpy(q).to(dev)
    phi, force, e = f.evaluate(tq)
    phi2, _, _ = f.evaluate(tq, want_force=False, want_energy=False)
    _, force3, _ = f.evaluate(tq, want_phi=False, want_energy=False)
    _, _, e4 = f.evaluate(-tq, want_phi=False, want_force=False)
    assert torch.equal(phi, phi2) and torch.equal(force, force3) and torch.equal(e, e4)
    assert f.check() == 0
    f.close()


def test_work_counts():
    import torch
    log("[api] work counts")
    pos, q = W.SMALL.make()
    f = B.FMM(torch.from_numpy(pos).to("cuda:0"), p=4, depth=3)
    m2l, p2p = B.fmm_plan_work(f.plan)
    f.close()
    cells, _, _ = oracle.leaf_cells(pos, 3)
    # independent count from the leaf cells
    occ = np.zeros((8, 8, 8), dtype=np.int64)
    np.add.at(occ, tuple(cells.T), 1)
    exp_p2p = 0
    for x, y, z in zip(*np.nonzero(occ)):
        sl = occ[max(x - 1, 0):x + 2, max(y - 1, 0):y + 2, max(z - 1, 0):z + 2].sum()
        exp_p2p += occ[x, y, z] * (sl - 1)
    assert p2p == exp_p2p
    exp_m2l = 0
    for level in (2, 3):
        nb = 1 << level
        o = occ.reshape(nb, 8 // nb, nb, 8 // nb, nb, 8 // nb).sum(axis=(1, 3, 5))
        boxes = np.argwhere(o > 0)
        for t in boxes:
            d = np.abs(boxes - t).max(axis=1)
            pd = np.abs(boxes // 2 - t // 2).max(axis=1)
            exp_m2l += int(((d > 1) & (pd <= 1)).sum())
    assert m2l == exp_m2l


def test_profile_phases():
    # The M2L phase times the M2L kernel alone (once per evaluation); the
    # split forms record their multipole split as a phase of its own.
    import torch
    pos, q = W.uniform_gauss(20000, 41)
    dev = torch.device("cuda:0")
    tp, tq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
    for prec, kind, split in ((B.FMM_PREC_MIXED, B.FMM_M2L_F16X2, 1), (B.FMM_PREC_MIXED, B.FMM_M2L_F32, 0),
                              (B.FMM_PREC_FP64, B.FMM_M2L_AUTO, 0)):
        f = B.FMM(tp, p=6, depth=4, precision=prec, m2l_kind=kind)
        B.fmm_profile_enable(f.plan, True)
        f.evaluate(tq)
        rec = B.fmm_profile_read(f.plan)
        assert rec["m2l"][1] == 1 and rec["m2l"][0] > 0
        assert rec["split"][1] == split
        assert rec["p2p"][1] == 1 and rec["p2m"][1] == 1
        f.close()


# 2^17 charges on a depth-5 tree at p = 8: 304 M2L work-groups, so every XCD
# runs 22 whole groups before its 16 split tail groups (cases with at most 128
# groups run every group split).  4,096 sampled targets against the oracle.
@pytest.mark.parametrize("precision,kind", [(B.FMM_PREC_FP64, B.FMM_M2L_AUTO),
                                            (B.FMM_PREC_MIXED, B.FMM_M2L_F32),
                                            (B.FMM_PREC_MIXED, B.FMM_M2L_BF16X3),
                                            (B.FMM_PREC_MIXED, B.FMM_M2L_F16X2)])
def test_depth5_whole_groups_sampled(precision, kind):
    log(f"[depth5] precision {precision} m2l {kind}")
    pos, q = W.uniform_gauss(1 << 17, 34)
    phi, force, e, _ = run_gpu(pos, q, 5, 8, precision=precision, m2l_kind=kind)
    t = np.arange(0, 1 << 17, 32)
    phi_o, force_o, _ = oracle.fmm(pos, q, 5, 8, targets=t)
    tol = 1e-12 if precision == B.FMM_PREC_FP64 else 1e-5
    assert_close(phi[t], phi_o, tol, what="phi")
    assert_close(force[t], force_o, tol, what="force")


@pytest.mark.parametrize("kw", [dict(p=6, depth=4, precision=B.FMM_PREC_FP64),
                                dict(p=8, depth=4, precision=B.FMM_PREC_MIXED),
                                dict(p=6, depth=6, precision=B.FMM_PREC_MIXED, leaf_max=16)],
                         ids=["fp64", "mixed-f16", "adaptive-mixed"])
def test_replan_equals_fresh_plan(kw):
    """fmm_replan (new positions, the operator tables kept) gives bitwise the
    result of a fresh fmm_plan for those positions."""
    import torch
    log(f"[api] replan {kw}")
    dev = torch.device("cuda:0")
    pos_a, q = W.uniform_gauss(20000, 81)
    pos_b, _ = W.uniform_gauss(20000, 82)
    tb, tq = torch.from_numpy(pos_b).to(dev), torch.from_numpy(q).to(dev)
    f = B.FMM(torch.from_numpy(pos_a).to(dev), **kw)
    f.evaluate(tq)
    B.fmm_replan(f.plan, tb)
    a = f.evaluate(tq)
    assert f.check() == 0
    g = B.FMM(tb, **kw)
    b = g.evaluate(tq)
    assert g.check() == 0
    for x, y in zip(a, b):
        assert torch.equal(x, y)
    f.close()
    g.close()


@pytest.mark.parametrize("prec", [B.FMM_PREC_MIXED, B.FMM_PREC_FP64], ids=["mixed", "fp64"])
def test_uniform_replan_and_evaluate_replay_as_one_graph(prec):
    """On the uniform tree fmm_replan and fmm_evaluate enqueue kernels only (no
    read-back, no memset node): the tree build for new positions and the
    evaluation are captured together as one hipGraph.  The positions are
    rewritten in place between replays, with unrelated eager work in between;
    every replay equals the eager replan + evaluate of those positions
    bitwise."""
    import torch
    dev = torch.device("cuda:0")
    pos, q = W.uniform_gauss(50_000, 141)
    rng = np.random.default_rng(142)
    pos2 = np.clip(pos + 0.01 * rng.standard_normal(pos.shape), 0.0, np.nextafter(1.0, 0.0))
    tp = torch.from_numpy(pos).to(dev)
    tq = torch.from_numpy(q).to(dev)
    f = B.FMM(tp, p=6, depth=4, precision=prec)
    n = len(q)
    out = [torch.empty(n, dtype=torch.float64, device=dev), torch.empty((n, 3), dtype=torch.float64, device=dev),
           torch.empty(1, dtype=torch.float64, device=dev)]
    ref = {}
    for name, P in (("a", pos), ("b", pos2)):
        tp.copy_(torch.from_numpy(P))
        B.fmm_replan(f.plan, tp)
        B.fmm_evaluate(f.plan, tq, *out)
        torch.cuda.synchronize()
        ref[name] = [o.clone() for o in out]
    assert not torch.equal(ref["a"][0], ref["b"][0])
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):  # warm-up on the capture stream
        B.fmm_replan(f.plan, tp)
        B.fmm_evaluate(f.plan, tq, *out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.fmm_replan(f.plan, tp)
        B.fmm_evaluate(f.plan, tq, *out)
    for rep, (name, P) in enumerate((("a", pos), ("b", pos2), ("a", pos))):
        tp.copy_(torch.from_numpy(P))
        for o in out:
            o.zero_()
        _ = (tq * 2.0).sum()  # unrelated eager work between replays
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(out, ref[name]):
            assert torch.equal(o, r), (rep, name)
    assert f.check() == 0
    f.close()
