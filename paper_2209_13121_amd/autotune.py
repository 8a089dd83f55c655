"""Autotuner: the fastest mixed-precision configuration that meets the accuracy gate.

For a given charge set and tree family it searches
  * the tree's leaf capacity (``leaf_max`` of an adaptive tree, or the depth
    of a uniform one), the knob that trades near-field (P2P) against far-field
    (M2L) work;
  * the M2L form (scaled split FP16, split BF16, FP32);
  * the schedule of the passes (``fmm_plan_set_schedule``): the adaptive P2P
    as one wave per box or as a persistent launch over a cost-ordered
    work-list; how many tail work-groups per XCD the split M2L forms run in
    four parts, or (the FP16 form at p <= 8) the M2L as a persistent launch
    over per-XCD tile counters;
  * then, for the best candidate on an adaptive tree, the P2P tile (sources
    staged in LDS at a time).
Every candidate is measured on the GPU through the C ABI, the way the
benchmark runs a step: one plan, then fmm_replan + fmm_evaluate timed with HIP
events on the launch stream (median of ``reps``).  The gate is the library's:
relative energy error <= 1e-6 and relative RMS force error <= 1e-5 against the
FP64 result of the same tree; a caller may add a check of its own (e.g.
against an independent reference on sampled systems) through ``reference``.

``select`` holds the decision rule alone (no GPU), so it can be tested on the
host.
"""
from dataclasses import dataclass, field

from . import binding as B

KINDS = ("F16X2", "BF16X3", "F32")
SPLIT_KINDS = ("F16X2", "BF16X3", "BF16X2")
# schedule values searched (key -> values); the first value is the default
SCHEDULES = {"p2p_persistent": (0, 1), "m2l_split": (16, 8, 0)}
_SCHED_KEY = {"p2p_persistent": B.FMM_SCHED_P2P_PERSISTENT, "m2l_split": B.FMM_SCHED_M2L_SPLIT,
              "m2l_persistent": B.FMM_SCHED_M2L_PERSISTENT, "p2p_tile": B.FMM_SCHED_P2P_TILE}
P2P_TILES = (128, 256, 512)  # sources per staged P2P tile; the first is the mixed default
WIDE_PMAX = 8  # the FP16 form's persistent M2L runs up to this order


@dataclass
class Result:
    tree: dict                 # leaf_max / depth of the candidate tree
    kind: str                  # M2L form
    ms: float                  # median replan + evaluate time
    energy_err: float          # relative to FP64 on the same tree
    force_err: float           # relative RMS, same reference
    schedule: dict = field(default_factory=dict)
    extra: dict = field(default_factory=dict)
    reference_ok: bool = True  # the caller's own check, when given

    def meets(self, gate_e, gate_f):
        return self.energy_err <= gate_e and self.force_err <= gate_f and self.reference_ok


def select(results, gate_e=1e-6, gate_f=1e-5):
    """The fastest result within the gate (ties: the earlier one); None when
    no candidate meets it."""
    best = None
    for r in results:
        if r.meets(gate_e, gate_f) and (best is None or r.ms < best.ms):
            best = r
    return best


def schedules_for(tree, kind, p=None):
    """The schedule candidates that apply to a tree, an M2L form and order p:
    the adaptive tree's two P2P forms, times the split forms' tail splits and,
    for the FP16 form at p <= WIDE_PMAX, the persistent M2L."""
    p2p = [{"p2p_persistent": v} for v in SCHEDULES["p2p_persistent"]] if tree.get("leaf_max", 0) > 0 else [{}]
    m2l = [{"m2l_split": v} for v in SCHEDULES["m2l_split"]] if kind in SPLIT_KINDS else [{}]
    if kind == "F16X2" and p is not None and p <= WIDE_PMAX:
        m2l.append({"m2l_persistent": 1})
    return [dict(**a, **b) for a in p2p for b in m2l]


def apply_schedule(plan, schedule):
    for k, v in schedule.items():
        B.fmm_plan_set_schedule(plan, _SCHED_KEY[k], v)


def _time(torch, cfg, n, pos, q, ws, stream, reps, schedule):
    """Median ms of replan + evaluate after one plan, and the last outputs."""
    phi = torch.empty(n, dtype=torch.float64, device=pos.device)
    force = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    energy = torch.empty(1, dtype=torch.float64, device=pos.device)
    plan = B.fmm_plan(cfg, n, pos, ws, stream)
    apply_schedule(plan, schedule)
    times = []
    for r in range(reps + 1):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(stream)
        B.fmm_replan(plan, pos, stream)
        B.fmm_evaluate(plan, q, phi, force, energy, stream)
        t1.record(stream)
        torch.cuda.synchronize()
        if r:  # the first run warms up
            times.append(t0.elapsed_time(t1))
    st = B.fmm_check(plan)
    B.fmm_destroy(plan)
    if st != 0:
        raise B.FMMError(st, "autotune candidate")
    times.sort()
    return times[len(times) // 2], phi, force, float(energy.cpu()[0])


def tune(pos, q, p, trees, kinds=KINDS, lo=(0.0, 0.0, 0.0), side=1.0, batch_level=0, reps=5,
         gate_e=1e-6, gate_f=1e-5, stream=None, search_schedules=True, reference=None):
    """Search ``trees`` x ``kinds`` x schedules (each tree a dict of
    make_config keywords, e.g. {"depth": 8, "leaf_max": 64} or {"depth": 6})
    for device tensors pos, q.  ``reference(tree, phi, force, energy) -> bool``,
    if given, is a further check every accepted candidate must pass.  Returns
    (best Result or None, all Results)."""
    import torch
    n = q.numel()
    stream = stream or torch.cuda.current_stream()
    results = []
    refs = {}  # tree -> the FP64 forces and energy of that tree

    def run(tree, kind, scheds):
        f64, e64, ms64 = refs[tuple(sorted(tree.items()))]
        fnorm = torch.linalg.vector_norm(f64)
        cfg = B.make_config(p=p, precision=B.FMM_PREC_MIXED, m2l_kind=getattr(B, "FMM_M2L_" + kind),
                            lo=lo, side=side, batch_level=batch_level, **tree)
        ws = torch.empty(B.fmm_workspace_size(cfg, n), dtype=torch.uint8, device=pos.device)
        for sched in scheds:
            ms, phi, f, e = _time(torch, cfg, n, pos, q, ws, stream, reps, sched)
            r = Result(tree=dict(tree), kind=kind, ms=ms, energy_err=abs(e - e64) / abs(e64),
                       force_err=float(torch.linalg.vector_norm(f - f64) / fnorm),
                       schedule=dict(sched), extra={"fp64_ms": ms64})
            if reference is not None and r.meets(gate_e, gate_f):
                r.reference_ok = bool(reference(tree, phi, f, e))
            results.append(r)
        del ws

    for tree in trees:
        ref_cfg = B.make_config(p=p, precision=B.FMM_PREC_FP64, lo=lo, side=side,
                                batch_level=batch_level, **tree)
        ws = torch.empty(B.fmm_workspace_size(ref_cfg, n), dtype=torch.uint8, device=pos.device)
        ms64, _, f64, e64 = _time(torch, ref_cfg, n, pos, q, ws, stream, 1, {})
        del ws
        refs[tuple(sorted(tree.items()))] = (f64, e64, ms64)
        for kind in kinds:
            run(tree, kind, schedules_for(tree, kind, p) if search_schedules else [{}])
        torch.cuda.empty_cache()
    best = select(results, gate_e, gate_f)
    # then the P2P tile of the best candidate (adaptive trees: the per-leaf kernels)
    if search_schedules and best is not None and best.tree.get("leaf_max", 0) > 0:
        run(best.tree, best.kind, [dict(best.schedule, p2p_tile=t) for t in P2P_TILES[1:]])
        best = select(results, gate_e, gate_f)
    return best, results
