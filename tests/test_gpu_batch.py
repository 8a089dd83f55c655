"""GPU parity of a batch of independent systems (adaptive tree with
batch_level > 0) through the C ABI, and hipGraph capture of the evaluation.

* FP64: every system of the batch against the oracle's adaptive FMM of that
  system alone, its cell as the root cube (same tree below the batch level):
  phi and F per particle to 1e-12, the energy as the sum over systems, and the
  P2P and M2L pair counts as sums of the per-system counts, exactly.
* Mixed: the same comparison within the gate (E 1e-6, RMS F 1e-5).
* One plan's evaluation captured in a hipGraph (torch.cuda.CUDAGraph) and
  replayed three times, with eager work in between: every replay equals the
  eager evaluation bitwise.
* The batch workload at full size (256 systems, 4.04e6 charges, p = 6): FP64
  against the oracle on sampled systems; mixed against FP64.
"""
import numpy as np
import pytest

import oracle
from gpu_util import assert_close, B, log, rel, run_gpu
from paper_2209_13121_amd import workloads as W

pytestmark = pytest.mark.gpu


def small_batch():
    rng = np.random.default_rng(51)
    pos, q, counts = W.batched_systems(10, 52, n_min=150, n_max=3000, grid=4)
    return pos, q, counts


def oracle_per_system(pos, q, counts, leaf_max, rel_depth, p, grid):
    phi = np.empty(len(q))
    force = np.empty((len(q), 3))
    e = 0.0
    pairs = {"p2p_pairs": 0, "m2l_pairs": 0}
    start = 0
    for k, nk in enumerate(counts):
        sl = slice(start, start + nk)
        cell = (k % grid, (k // grid) % grid, k // (grid * grid))
        ph, f, ek, st = oracle.fmm_adaptive(pos[sl], q[sl], leaf_max, rel_depth, p, lo=cell, side=1.0)
        phi[sl], force[sl] = ph, f
        e += ek
        for key in pairs:
            pairs[key] += st[key]
        start += nk
    return phi, force, e, pairs


def run_batch(pos, q, cap, p, prec, leaf_max, level, grid, stats=None, kind=B.FMM_M2L_AUTO):
    return run_gpu(pos, q, cap, p, prec, lo=(0.0, 0.0, 0.0), side=float(grid), leaf_max=leaf_max,
                   stats=stats, m2l_kind=kind, batch_level=level)


@pytest.mark.parametrize("prec", [B.FMM_PREC_FP64, B.FMM_PREC_MIXED])
def test_batch_matches_per_system_oracle(prec):
    pos, q, counts = small_batch()
    phi_o, f_o, e_o, pairs = oracle_per_system(pos, q, counts, 16, 4, 4, 4)
    st = {}
    phi, force, e, _ = run_batch(pos, q, 6, 4, prec, 16, 2, 4, stats=st)
    log(f"[batch] prec {prec}: stats {st}")
    assert st["p2p_pairs"] == pairs["p2p_pairs"]
    assert st["m2l_pairs"] == pairs["m2l_pairs"]
    tol_phi, tol_f, tol_e = (1e-12, 1e-12, 1e-12) if prec == B.FMM_PREC_FP64 else (1e-5, 1e-5, 1e-6)
    assert_close(phi, phi_o, tol_phi, what="phi")
    assert_close(force, f_o, tol_f, what="force")
    assert abs(e - e_o) <= tol_e * abs(e_o)


def test_many_tiny_systems_depth_at_batch_level():
    # 512 systems of 2 charges, one per cell of level 3, depth cap = batch
    # level = 3: every box above level 3 holding a charge is divided although
    # it holds fewer than leaf_max charges, so the workspace bound on the
    # number of boxes must count such boxes (min(8^l, n) per level).  Each
    # system is then its own leaf: the result is the direct sum per system.
    rng = np.random.default_rng(53)
    grid = 8
    cells = np.array([(k % grid, (k // grid) % grid, k // (grid * grid)) for k in range(512)],
                     dtype=np.float64)
    pos = np.repeat(cells, 2, axis=0) + rng.random((1024, 3))
    q = np.tile([1.0, -1.0], 512)
    st = {}
    phi, force, e, _ = run_batch(pos, q, 3, 4, B.FMM_PREC_FP64, 64, 3, grid, stats=st)
    assert st["boxes"] == 1 + 8 + 64 + 512 and st["leaves"] == 512
    d = pos[0::2] - pos[1::2]
    r = np.sqrt((d * d).sum(axis=1))
    phi_d = np.empty(1024)
    phi_d[0::2], phi_d[1::2] = -1.0 / r, 1.0 / r
    f_d = np.empty((1024, 3))
    f_d[0::2] = -(d / r[:, None] ** 3)  # F_i = q_i q_j (x_i - x_j) / r^3, q_i q_j = -1
    f_d[1::2] = d / r[:, None] ** 3
    assert_close(phi, phi_d, 1e-13, what="phi")
    assert_close(force, f_d, 1e-13, what="force")
    assert abs(e - (-1.0 / r).sum()) <= 1e-13 * abs((1.0 / r).sum())


@pytest.mark.parametrize("prec", [B.FMM_PREC_MIXED, B.FMM_PREC_FP64])
def test_schedules_give_the_same_result(prec):
    """The persistent work-list P2P and every P2P tile equal the per-box
    launch bitwise; the M2L tail split only reorders a sum (within rounding);
    bad keys and values are refused."""
    import torch
    pos, q, counts = small_batch()
    dev = torch.device("cuda:0")
    tp, tq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
    f = B.FMM(tp, p=4, depth=6, precision=prec, lo=(0.0, 0.0, 0.0), side=4.0, leaf_max=16,
              batch_level=2)
    a = f.evaluate(tq)
    B.fmm_plan_set_schedule(f.plan, B.FMM_SCHED_P2P_PERSISTENT, 1)
    b = f.evaluate(tq)
    B.fmm_replan(f.plan, tp)  # the schedule survives a re-plan
    c = f.evaluate(tq)
    assert f.check() == 0
    for x, y, z in zip(a, b, c):
        assert torch.equal(x, y) and torch.equal(x, z)
    for tile in (128, 256, 512):  # the P2P tile: the same sums in the same order
        B.fmm_plan_set_schedule(f.plan, B.FMM_SCHED_P2P_TILE, tile)
        d = f.evaluate(tq)
        for x, y in zip(a, d):
            assert torch.equal(x, y)
    B.fmm_plan_set_schedule(f.plan, B.FMM_SCHED_P2P_TILE, 256)
    for split in (0, 8):
        B.fmm_plan_set_schedule(f.plan, B.FMM_SCHED_M2L_SPLIT, split)
        d = f.evaluate(tq)
        assert_close(d[0].cpu().numpy(), a[0].cpu().numpy(), 1e-12 if prec == B.FMM_PREC_FP64 else 1e-6,
                     what=f"phi split {split}")
    with pytest.raises(B.FMMError):
        B.fmm_plan_set_schedule(f.plan, 7, 0)
    with pytest.raises(B.FMMError):
        B.fmm_plan_set_schedule(f.plan, B.FMM_SCHED_M2L_SPLIT, 17)
    with pytest.raises(B.FMMError):
        B.fmm_plan_set_schedule(f.plan, B.FMM_SCHED_P2P_TILE, 300)
    f.close()
    u = B.FMM(tp[:1000].contiguous(), p=4, depth=3, precision=prec, lo=(0.0, 0.0, 0.0), side=4.0)
    with pytest.raises(B.FMMError) as ei:  # the work-list exists for adaptive trees only
        B.fmm_plan_set_schedule(u.plan, B.FMM_SCHED_P2P_PERSISTENT, 1)
    assert ei.value.status == 6
    u.close()


@pytest.mark.parametrize("tree", ["uniform", "adaptive"])
def test_persistent_m2l_equals_unsplit(tree):
    """The persistent M2L (FP16 form, p <= 8) sums every tile as the unsplit
    launch does: bitwise equal to FMM_SCHED_M2L_SPLIT 0, on a uniform tree
    with full tiles (levels 4-5) and on the batch forest; refused where the
    form does not run."""
    import torch
    dev = torch.device("cuda:0")
    if tree == "uniform":
        pos, q = W.uniform_gauss(200_000, 131)
        kw = dict(p=8, depth=5)
    else:
        pos, q, _ = small_batch()
        kw = dict(p=6, depth=6, lo=(0.0, 0.0, 0.0), side=4.0, leaf_max=16, batch_level=2)
    tp, tq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
    f = B.FMM(tp, precision=B.FMM_PREC_MIXED, m2l_kind=B.FMM_M2L_F16X2, **kw)
    B.fmm_plan_set_schedule(f.plan, B.FMM_SCHED_M2L_SPLIT, 0)
    a = f.evaluate(tq)
    B.fmm_plan_set_schedule(f.plan, B.FMM_SCHED_M2L_PERSISTENT, 1)
    b = f.evaluate(tq)
    B.fmm_replan(f.plan, tp)  # the schedule survives a re-plan
    c = f.evaluate(tq)
    assert f.check() == 0
    for x, y, z in zip(a, b, c):
        assert torch.equal(x, y) and torch.equal(x, z)
    f.close()
    g = B.FMM(tp, precision=B.FMM_PREC_MIXED, m2l_kind=B.FMM_M2L_BF16X3, **kw)
    with pytest.raises(B.FMMError) as ei:
        B.fmm_plan_set_schedule(g.plan, B.FMM_SCHED_M2L_PERSISTENT, 1)
    assert ei.value.status == 6
    g.close()


def test_graph_replay_equals_eager():
    import torch
    pos, q, counts = small_batch()
    dev = torch.device("cuda:0")
    tp, tq = torch.from_numpy(pos).to(dev), torch.from_numpy(q).to(dev)
    for prec in (B.FMM_PREC_MIXED, B.FMM_PREC_FP64):
        f = B.FMM(tp, p=4, depth=6, precision=prec, lo=(0.0, 0.0, 0.0), side=4.0, leaf_max=16,
                  batch_level=2)
        phi0, force0, e0 = f.evaluate(tq)
        torch.cuda.synchronize()
        phi = torch.empty_like(phi0)
        force = torch.empty_like(force0)
        e = torch.empty_like(e0)
        g = torch.cuda.CUDAGraph()
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            B.fmm_evaluate(f.plan, tq, phi, force, e)  # warm-up on the capture stream
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            B.fmm_evaluate(f.plan, tq, phi, force, e)
        for rep in range(3):
            phi.zero_()
            force.zero_()
            e.zero_()
            _ = (tq * 2.0).sum()  # unrelated eager work between replays
            g.replay()
            torch.cuda.synchronize()
            assert torch.equal(phi, phi0) and torch.equal(force, force0) and torch.equal(e, e0), rep
        f.close()


@pytest.fixture(scope="module")
def batch_full():
    wl = W.BATCH
    pos, q, counts = wl.make()
    return wl, pos, q, counts


def test_batch_full_size(batch_full):
    wl, pos, q, counts = batch_full
    grid = 1 << wl.batch_level
    log(f"[batch full] {wl.name}: {len(q)} charges")
    phi64, f64, e64, _ = run_batch(pos, q, wl.max_depth, wl.p, B.FMM_PREC_FP64, wl.leaf_max,
                                   wl.batch_level, grid)
    phim, fm, em, _ = run_batch(pos, q, wl.max_depth, wl.p, B.FMM_PREC_MIXED, wl.leaf_max,
                                wl.batch_level, grid)
    assert abs(em - e64) <= 1e-6 * abs(e64)
    assert_close(fm, f64, 1e-5, what="fm")
    # three systems (the smallest, a middle one, the largest) against the oracle
    starts = np.concatenate([[0], np.cumsum(counts)])
    for k in (int(np.argmin(counts)), len(counts) // 2, int(np.argmax(counts))):
        sl = slice(starts[k], starts[k + 1])
        cell = (k % grid, (k // grid) % grid, k // (grid * grid))
        ph, f, ek, _ = oracle.fmm_adaptive(pos[sl], q[sl], wl.leaf_max, wl.max_depth - wl.batch_level,
                                           wl.p, lo=cell, side=1.0)
        log(f"[batch full] system {k} ({counts[k]} charges)")
        assert_close(phi64[sl], ph, 1e-12, what="phi64")
        assert_close(f64[sl], f, 1e-12, what="f64")
