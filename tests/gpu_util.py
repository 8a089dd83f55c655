"""Helpers shared by the GPU tests: run the HIP library through its C ABI on
torch device tensors and compare with the CPU oracle."""
import math
import sys

import numpy as np

from paper_2209_13121_amd import binding as B


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def device():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("no HIP device")
    return torch.device("cuda:0")


def run_gpu(pos, q, depth, p, precision=B.FMM_PREC_FP64, lo=(0.0, 0.0, 0.0), side=1.0,
            check=True, m2l_kind=B.FMM_M2L_AUTO, leaf_max=0, stats=None, batch_level=0):
    """Plan + evaluate on the GPU; returns numpy (phi, force, energy, status).
    leaf_max > 0: adaptive tree (depth = its cap); a dict passed as stats
    receives the tree statistics."""
    import torch
    dev = device()
    tp = torch.from_numpy(np.ascontiguousarray(pos, dtype=np.float64)).to(dev)
    tq = torch.from_numpy(np.ascontiguousarray(q, dtype=np.float64)).to(dev)
    f = B.FMM(tp, p=p, depth=depth, precision=precision, lo=lo, side=side, m2l_kind=m2l_kind,
              leaf_max=leaf_max, batch_level=batch_level)
    phi, force, energy = f.evaluate(tq)
    st = f.check()
    torch.cuda.synchronize()
    out = (phi.cpu().numpy(), force.cpu().numpy(), float(energy.cpu().numpy()[0]), st)
    if stats is not None and leaf_max > 0:
        stats.update(B.fmm_plan_tree_stats(f.plan))
    f.close()
    if check and st != 0:
        raise B.FMMError(st, "device flag")
    return out


def rel(a, b):
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / nb) if nb > 0 else float(np.linalg.norm(a - b))


def energy_rel(e, e_ref):
    return abs(e - e_ref) / abs(e_ref)


def half_sum_q_phi(q, phi):
    return 0.5 * math.fsum(np.asarray(q) * np.asarray(phi))


def elem(a, b):
    """Largest per-particle error, relative to the particle's own value and
    at least to the RMS of the reference:
    max_i |a_i - b_i| / max(|b_i|, sqrt(mean_j |b_j|^2)), |.| the Euclidean
    norm of a row (a force) or the absolute value (a potential).  (A particle
    with a close neighbour carries a force many times the RMS, and its
    rounding is relative to its own size; a wrong tile or box gives an error of
    the order of the far field, caught against either denominator.)"""
    a, b = np.asarray(a, dtype=float), np.asarray(b, dtype=float)
    d = (a - b).reshape(len(b), -1)
    r = b.reshape(len(b), -1)
    if not len(b):
        return 0.0
    mag = np.sqrt(np.sum(r * r, axis=1))
    rms = math.sqrt(float(np.mean(mag * mag)))
    den = np.maximum(mag, rms) if rms > 0 else np.ones_like(mag)
    return float((np.sqrt(np.sum(d * d, axis=1)) / den).max())


def assert_close(a, b, norm, elem_tol=None, what=""):
    """Normwise relative error <= norm and per-particle error <= elem_tol
    (elem above; default 1e-10 beside an FP64 rounding bound, else 10 x norm),
    so that one bad box cannot hide under the norm."""
    if elem_tol is None:
        elem_tol = 1e-10 if norm <= 1e-11 else 10.0 * norm
    r, e = rel(a, b), elem(a, b)
    if what:
        log(f"  {what}: normwise {r:.2e} (<= {norm:.0e}), per-particle {e:.2e} (<= {elem_tol:.0e})")
    assert r <= norm, f"{what} normwise {r:.3e} > {norm:.1e}"
    assert e <= elem_tol, f"{what} per-particle {e:.3e} > {elem_tol:.1e}"
