"""GPU test of fmm_evaluate_static, the entry point that allocates nothing
(its workspace is the library's device scratch array), through the C ABI.

Each call's potentials, forces and energy must equal, bitwise, those of
fmm_plan + fmm_evaluate on a workspace of the caller's (the same kernels on the
same layout, every sum in a fixed order), on two calls in a row, the second
with a smaller input; a plan larger than the scratch array is refused.
"""
import numpy as np
import pytest

from gpu_util import B, device, log
from paper_2209_13121_amd import workloads as W

pytestmark = pytest.mark.gpu


def planned(pos, q, cfg):
    """fmm_plan + fmm_evaluate on a caller workspace."""
    import torch
    n = len(q)
    ws = torch.empty(B.fmm_workspace_size(cfg, n), dtype=torch.uint8, device=pos.device)
    plan = B.fmm_plan(cfg, n, pos, ws)
    phi = torch.empty(n, dtype=torch.float64, device=pos.device)
    force = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    e = torch.empty(1, dtype=torch.float64, device=pos.device)
    B.fmm_evaluate(plan, q, phi, force, e)
    assert B.fmm_check(plan) == 0
    B.fmm_destroy(plan)
    return phi, force, e


def static(pos, q, cfg):
    import torch
    n = len(q)
    phi = torch.full((n,), np.nan, dtype=torch.float64, device=pos.device)
    force = torch.full((n, 3), np.nan, dtype=torch.float64, device=pos.device)
    e = torch.full((1,), np.nan, dtype=torch.float64, device=pos.device)
    plan = B.fmm_evaluate_static(cfg, n, pos, q, phi, force, e)
    assert B.fmm_check(plan) == 0
    B.fmm_destroy(plan)  # only waits: the plan is the library's
    return phi, force, e


CASES = [
    # (name, inputs, config): each second case smaller than the first
    ("mixed-n30000-L4-p8", lambda: W.uniform_gauss(30000, 101),
     dict(p=8, depth=4, precision=B.FMM_PREC_MIXED)),
    ("fp64-n4096-L3-p4", lambda: W.uniform_pm1(4096, 102), dict(p=4, depth=3)),
    ("adaptive-mixed-n3000-cap5-p10", lambda: W.molecular_clusters(1000, 103)[:2],
     dict(p=10, depth=5, precision=B.FMM_PREC_MIXED, leaf_max=24, side=0.0)),
    ("adaptive-fp64-n1500-cap5-p6", lambda: W.molecular_clusters(500, 104)[:2],
     dict(p=6, depth=5, leaf_max=24, side=0.0)),
]


@pytest.mark.parametrize("pair", [(0, 1), (2, 3), (0, 3)], ids=lambda p: f"{p[0]}-then-{p[1]}")
def test_static_equals_planned_on_two_calls(pair):
    import torch
    dev = device()
    for k in pair:
        name, make, kw = CASES[k]
        log(f"[no-alloc] {name}")
        pos_np, q_np = make()
        pos = torch.from_numpy(np.ascontiguousarray(pos_np)).to(dev)
        q = torch.from_numpy(np.ascontiguousarray(q_np)).to(dev)
        cfg = B.make_config(**kw)
        assert B.fmm_workspace_size(cfg, len(q_np)) <= B.FMM_STATIC_SCRATCH_BYTES
        a = planned(pos, q, cfg)
        b = static(pos, q, cfg)
        torch.cuda.synchronize()
        for x, y in zip(a, b):
            assert torch.equal(x, y)


def test_static_refuses_a_plan_beyond_the_scratch_array():
    import torch
    dev = device()
    pos_np, q_np = W.uniform_gauss(1 << 17, 105)
    cfg = B.make_config(p=8, depth=5, precision=B.FMM_PREC_MIXED)
    assert B.fmm_workspace_size(cfg, len(q_np)) > B.FMM_STATIC_SCRATCH_BYTES
    pos = torch.from_numpy(pos_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    phi = torch.zeros(len(q_np), dtype=torch.float64, device=dev)
    with pytest.raises(B.FMMError) as ei:
        B.fmm_evaluate_static(cfg, len(q_np), pos, q, phi)
    assert ei.value.status == 2  # FMM_E_WORKSPACE
    assert int(torch.count_nonzero(phi)) == 0
