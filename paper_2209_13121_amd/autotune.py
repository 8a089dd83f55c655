"""Autotuner: the fastest mixed-precision configuration that meets the accuracy gate.

For a given charge set and tree family it searches the M2L form (scaled split
FP16, split BF16, FP32) and the tree's leaf capacity (``leaf_max`` of an
adaptive tree, or the depth of a uniform one), the knob that trades near-field
(P2P) against far-field (M2L) work.  Every candidate is measured on the GPU
through the C ABI: plan + evaluate timed with HIP events on the launch stream
(median of ``reps``), and its energy and forces compared with the FP64 result
of the same tree.  The gate is the library's: relative energy error <= 1e-6 and
relative RMS force error <= 1e-5 against FP64 of the same tree.

``select`` holds the decision rule alone (no GPU), so it can be tested on the
host.
"""
from dataclasses import dataclass, field

from . import binding as B

KINDS = ("F16X2", "BF16X3", "F32")


@dataclass
class Result:
    tree: dict                 # leaf_max / depth of the candidate tree
    kind: str                  # M2L form
    ms: float                  # median plan + evaluate time
    energy_err: float          # relative to FP64 on the same tree
    force_err: float           # relative RMS, same reference
    extra: dict = field(default_factory=dict)

    def meets(self, gate_e, gate_f):
        return self.energy_err <= gate_e and self.force_err <= gate_f


def select(results, gate_e=1e-6, gate_f=1e-5):
    """The fastest result within the gate (ties: the earlier one); None when
    no candidate meets it."""
    best = None
    for r in results:
        if r.meets(gate_e, gate_f) and (best is None or r.ms < best.ms):
            best = r
    return best


def _time(torch, cfg, n, pos, q, ws, stream, reps):
    """Median ms of plan + evaluate, and the outputs of the last run."""
    phi = torch.empty(n, dtype=torch.float64, device=pos.device)
    force = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    energy = torch.empty(1, dtype=torch.float64, device=pos.device)
    times = []
    for r in range(reps + 1):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        plan = B.fmm_plan(cfg, n, pos, ws, stream)
        B.fmm_evaluate(plan, q, phi, force, energy, stream)
        t1.record(stream)
        torch.cuda.synchronize()
        st = B.fmm_check(plan)
        B.fmm_destroy(plan)
        if st != 0:
            raise B.FMMError(st, "autotune candidate")
        if r:  # the first run warms up
            times.append(t0.elapsed_time(t1))
    times.sort()
    return times[len(times) // 2], phi, force, float(energy.cpu()[0])


def tune(pos, q, p, trees, kinds=KINDS, lo=(0.0, 0.0, 0.0), side=1.0, batch_level=0, reps=5,
         gate_e=1e-6, gate_f=1e-5, stream=None):
    """Search ``kinds`` x ``trees`` (each a dict of make_config keywords, e.g.
    {"depth": 8, "leaf_max": 64} or {"depth": 6}) for device tensors pos, q.
    Returns (best Result or None, all Results)."""
    import torch
    n = q.numel()
    stream = stream or torch.cuda.current_stream()
    results = []
    for tree in trees:
        ref_cfg = B.make_config(p=p, precision=B.FMM_PREC_FP64, lo=lo, side=side,
                                batch_level=batch_level, **tree)
        ws = torch.empty(B.fmm_workspace_size(ref_cfg, n), dtype=torch.uint8, device=pos.device)
        ms64, _, f64, e64 = _time(torch, ref_cfg, n, pos, q, ws, stream, 1)
        del ws
        fnorm = torch.linalg.vector_norm(f64)
        for kind in kinds:
            cfg = B.make_config(p=p, precision=B.FMM_PREC_MIXED, m2l_kind=getattr(B, "FMM_M2L_" + kind),
                                lo=lo, side=side, batch_level=batch_level, **tree)
            ws = torch.empty(B.fmm_workspace_size(cfg, n), dtype=torch.uint8, device=pos.device)
            ms, _, f, e = _time(torch, cfg, n, pos, q, ws, stream, reps)
            del ws
            results.append(Result(tree=dict(tree), kind=kind, ms=ms,
                                  energy_err=abs(e - e64) / abs(e64),
                                  force_err=float(torch.linalg.vector_norm(f - f64) / fnorm),
                                  extra={"fp64_ms": ms64}))
        torch.cuda.empty_cache()
    return select(results, gate_e, gate_f), results
