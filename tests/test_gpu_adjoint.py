"""GPU tests of the adjoint (fmm_backward and the torch.autograd.Function).

* dE/dq = phi and dE/dx = -F exactly (bitwise: the backward pass recomputes
  the same passes), scaled by the upstream gradient.
* Central finite differences of the oracle's FP64 FMM energy, on particles
  farther than the step from every box face, so that no difference crosses a
  face: computed in the test at a small size, and stored (h = 1e-4, 64
  coordinates and 64 charges) for the differentiation workload (2^19 charges).
* At the 2^19 size, mixed (FP32) forward: dE/dx against the oracle's direct-sum
  forces on 32,768 particles and against the oracle FMM, dE/dq against the
  oracle FMM potentials, on sampled particles.
"""
import numpy as np
import pytest

import oracle
from gpu_util import assert_close, B, log, rel
from paper_2209_13121_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev():
    import torch
    return torch.device("cuda:0")


def fd_candidates(pos, depth, h, min_nn):
    """Particles at least h from every face of their leaf (hence of every
    ancestor box) and at least min_nn from their nearest neighbour, so that a
    central difference with step h neither crosses a face nor suffers from the
    large third derivatives of a close pair."""
    from scipy.spatial import cKDTree
    u = pos * (1 << depth)
    frac = u - np.floor(u)
    away = np.all((frac > h * (1 << depth)) & (frac < 1 - h * (1 << depth)), axis=1)
    d, _ = cKDTree(pos).query(pos, k=2)
    return np.nonzero(away & (d[:, 1] > min_nn))[0]


@pytest.mark.parametrize("precision", [B.FMM_PREC_FP64, B.FMM_PREC_MIXED])
def test_backward_equals_forward_fields(precision):
    import torch
    log(f"[adjoint] backward vs forward, precision {precision}")
    pos, q = W.uniform_gauss(20000, 91)
    dev = _dev()
    f = B.FMM(torch.from_numpy(pos).to(dev), p=6, depth=4, precision=precision)
    tq = torch.from_numpy(q).to(dev)
    phi, force, e = f.evaluate(tq)
    g = torch.tensor([2.5], dtype=torch.float64, device=dev)
    dx = torch.empty((len(q), 3), dtype=torch.float64, device=dev)
    dq = torch.empty(len(q), dtype=torch.float64, device=dev)
    B.fmm_backward(f.plan, g, dx, dq)
    assert f.check() == 0
    assert torch.equal(dq, 2.5 * phi)
    assert torch.equal(dx, -2.5 * force)
    f.close()


def test_backward_requires_an_evaluation():
    import torch
    pos, q = W.uniform_gauss(1000, 92)
    f = B.FMM(torch.from_numpy(pos).to(_dev()), p=4, depth=3)
    g = torch.ones(1, dtype=torch.float64, device=_dev())
    with pytest.raises(B.FMMError) as ei:
        B.fmm_backward(f.plan, g, None, torch.empty(1000, dtype=torch.float64, device=_dev()))
    assert ei.value.status == 1
    f.close()


def test_autograd_against_oracle_finite_differences():
    import torch
    log("[adjoint] autograd vs FD of the oracle energy")
    depth, p, n, hfd = 3, 6, 4096, 1e-6
    pos, q = W.uniform_pm1(n, 93)
    dev = _dev()
    tp = torch.from_numpy(pos).to(dev).requires_grad_(True)
    tq = torch.from_numpy(q).to(dev).requires_grad_(True)
    e = B.fmm_energy(tp, tq, p=p, depth=depth)
    e.backward()
    gx, gq = tp.grad.cpu().numpy(), tq.grad.cpu().numpy()
    rng = np.random.default_rng(7)
    idx = rng.choice(fd_candidates(pos, depth, 2 * hfd, 0.03), 64, replace=False)
    for i in idx[:32]:
        a = rng.integers(3)
        pp, pm = pos.copy(), pos.copy()
        pp[i, a] += hfd
        pm[i, a] -= hfd
        fd = (oracle.fmm(pp, q, depth, p)[2] - oracle.fmm(pm, q, depth, p)[2]) / (2 * hfd)
        assert abs(fd - gx[i, a]) <= 1e-6 * max(1.0, abs(gx[i, a])), (i, a, fd, gx[i, a])
    hq = 1e-2  # E is quadratic in q: central differences are exact for any step
    for i in idx[32:]:
        qp, qm = q.copy(), q.copy()
        qp[i] += hq
        qm[i] -= hq
        fd = (oracle.fmm(pos, qp, depth, p)[2] - oracle.fmm(pos, qm, depth, p)[2]) / (2 * hq)
        assert abs(fd - gq[i]) <= 1e-8 * max(1.0, abs(gq[i])), (i, fd, gq[i])


def test_differentiation_workload():
    """2^19 +-1 charges, depth 6, p = 8, FP32 forward (mixed) with autograd:
    the differentiation protocol of the workload.
      * Central differences (h = 1e-4) of the FP64 oracle energy at 64
        (particle, axis) coordinates and 64 charges, stored by
        tests/golden/make_adjoint_fd.py (oracle only).  The coordinate
        differences carry an O(h^2) truncation, so each is also stored at h/2:
        the gradient must match the Richardson combination (4 D(h/2) - D(h)) / 3
        to the precision gate, and D(h) to its own estimated truncation.
      * Direct-sum forces on 32,768 sampled particles (FMM truncation at p = 8).
      * The oracle FMM on 512 sampled particles (the precision gate).
    The FP64 gradients go through the same stored differences."""
    import json
    import os
    import torch
    wl = W.ADJOINT
    log(f"[adjoint] {wl.name}")
    pos, q = wl.make()
    g = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                    "adjoint_fd.json")))
    assert g["workload"] == wl.name and g["h"] == 1e-4
    ix, ax = np.array(g["x_index"]), np.array(g["x_axis"])
    d_h, d_h2 = np.array(g["dE_dx_fd_h"]), np.array(g["dE_dx_fd_h_half"])
    rich = (4.0 * d_h2 - d_h) / 3.0
    trunc = np.abs(d_h - d_h2) * 4.0 / 3.0  # estimated truncation of D(h)
    rms_x = np.sqrt(np.mean(rich ** 2))
    iq, d_q = np.array(g["q_index"]), np.array(g["dE_dq_fd"])
    rms_q = np.sqrt(np.mean(d_q ** 2))
    dev = _dev()
    grads = {}
    for prec in (B.FMM_PREC_MIXED, B.FMM_PREC_FP64):
        tp = torch.from_numpy(pos).to(dev).requires_grad_(True)
        tq = torch.from_numpy(q).to(dev).requires_grad_(True)
        B.fmm_energy(tp, tq, p=wl.p, depth=wl.depth, precision=prec).backward()
        gx, gq = tp.grad.cpu().numpy(), tq.grad.cpu().numpy()
        grads[prec] = (gx, gq)
        tol = 2e-5 if prec == B.FMM_PREC_MIXED else 1e-6
        ex = np.abs(gx[ix, ax] - rich)
        log(f"  precision {prec}: dE/dx vs Richardson FD max {ex.max() / rms_x:.2e} of RMS; "
            f"vs D(h) max {np.max(np.abs(gx[ix, ax] - d_h) / (trunc + tol * rms_x)):.2f} of bound; "
            f"dE/dq vs FD max {np.max(np.abs(gq[iq] - d_q)) / rms_q:.2e} of RMS")
        assert np.all(ex <= tol * rms_x + 0.01 * trunc)
        assert np.all(np.abs(gx[ix, ax] - d_h) <= 1.5 * trunc + tol * rms_x)
        assert np.all(np.abs(gq[iq] - d_q) <= 10 * tol * rms_q)

    gx, gq = grads[B.FMM_PREC_MIXED]
    rng = np.random.default_rng(8)
    t = np.sort(rng.choice(wl.n, 32768, replace=False))
    log("  direct-sum forces on 32,768 particles (oracle)")
    _, f_dir, _ = oracle.direct(pos, q, targets=t)
    assert_close(-gx[t], f_dir, 1e-4, elem_tol=1e-2, what="dE/dx vs direct")  # FMM truncation at p = 8 plus FP32
    phi_o, f_o, _ = oracle.fmm(pos, q, wl.depth, wl.p, targets=t[:512])
    assert_close(-gx[t[:512]], f_o, 1e-5, what="dE/dx vs oracle FMM")
    assert_close(gq[t[:512]], phi_o, 1e-5, what="dE/dq vs oracle FMM")
