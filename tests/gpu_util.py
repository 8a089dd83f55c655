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
