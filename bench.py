"""Benchmark: FMM throughput on one MI355X (particles per second per evaluation).

Workload: 2^20 charges uniform in the unit cube, Gaussian charges shifted to
net zero (seed 1002), uniform octree of depth 6, expansion order p = 8.  One
step = fmm_replan (the tree build for the positions; the translation
operators, a function of p and the M2L form only, come from the first
fmm_plan) + fmm_evaluate (all passes, potentials, forces and energy) on
device-resident inputs.  Three variants are
timed the same way: mixed precision with the scaled split-FP16 M2L (the
library's default mixed form, the headline value), with the split-BF16 M2L,
with the FP32 M2L, and FP64; every energy is compared to the stored FP64
oracle energy.

Prints one JSON line.  ``--gpus N`` with N > 1 is refused: this build runs on
one GPU.
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "particles/s per FMM evaluation at 1e-6 rel. energy err, mixed vs FP64"
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6, "bf16": 2500.0, "f16": 2500.0}  # MI355X dense matrix peaks

# Timed variants: name -> (precision, m2l_kind, M2L kernel, its sources, dtype
# of the matrix-core work, piece products per FP32 product).
VARIANTS = {
    "mixed_bf16x3": ("MIXED", "BF16X3", "k_m2l_bf<8,3>",
                     ["paper_2209_13121_amd/csrc/m2l_bf16.hip", "paper_2209_13121_amd/csrc/m2l_common.h",
                      "paper_2209_13121_amd/csrc/bf16_split.h", "paper_2209_13121_amd/csrc/fmm_internal.h"],
                     "bf16", 6),
    "mixed_f16x2": ("MIXED", "F16X2", "k_m2l_w<8>",
                    ["paper_2209_13121_amd/csrc/m2l_bf16.hip", "paper_2209_13121_amd/csrc/m2l_common.h",
                     "paper_2209_13121_amd/csrc/bf16_split.h", "paper_2209_13121_amd/csrc/fmm_internal.h"],
                    "f16", 3),
    "mixed_f32": ("MIXED", "F32", "k_m2l<8,float>",
                  ["paper_2209_13121_amd/csrc/m2l.hip", "paper_2209_13121_amd/csrc/m2l_common.h",
                   "paper_2209_13121_amd/csrc/fmm_internal.h"],
                  "f32", 1),
    "fp64": ("FP64", "AUTO", "k_m2l<8,double>",
             ["paper_2209_13121_amd/csrc/m2l.hip", "paper_2209_13121_amd/csrc/m2l_common.h",
              "paper_2209_13121_amd/csrc/fmm_internal.h"],
             "f64", 1),
}
HEADLINE = "mixed_f16x2"  # the mixed form the library picks for FMM_M2L_AUTO


def traffic_summary(variant):
    return f"profiles/k_m2l_{variant}_uniform-gauss-n1048576-depth6-p8_hbm_counters.txt"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adaptive", action="store_true",
                    help="skip the adaptive-tree workload (10^6 three-site clusters)")
    ap.add_argument("--adaptive-only", action="store_true",
                    help="run only the adaptive-tree workload and print its JSON object")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the 256-system batch and print its JSON object")
    ap.add_argument("--cpu-sample-boxes", type=int, default=2,
                    help="level-1 boxes (1/8 of the domain each) whose particles the oracle evaluates")
    ap.add_argument("--p2p-only", action="store_true",
                    help="run only the near-field pass on the depth-4 tree (profiling runs)")
    ap.add_argument("--only", choices=sorted(VARIANTS), default=None,
                    help="time one variant only (profiling runs)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only copy MIB MiB device-to-device 5 times (HBM counter calibration) and exit")
    return ap.parse_args()


def copy_calibration(mib):
    """A plain device copy of known size: 5 launches, each reading and writing
    mib MiB, to scale the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * 2**20 // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_per_launch": n * 4, "launches": 5}), flush=True)


def graph_step(B, torch, pos, q, cfg, ws, steps, warmup):
    """The headline step (fmm_replan + fmm_evaluate; uniform tree: kernels
    only) captured once as a hipGraph and replayed: ms per replay (HIP events
    around the replays) and whether a replay equals the eager step bitwise."""
    n = q.numel()
    out = [torch.empty(n, dtype=torch.float64, device=pos.device),
           torch.empty((n, 3), dtype=torch.float64, device=pos.device),
           torch.empty(1, dtype=torch.float64, device=pos.device)]
    plan = B.fmm_plan(cfg, n, pos, ws)
    B.fmm_replan(plan, pos)
    B.fmm_evaluate(plan, q, *out)
    torch.cuda.synchronize()
    eager = [o.clone() for o in out]
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        B.fmm_replan(plan, pos)
        B.fmm_evaluate(plan, q, *out)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        B.fmm_replan(plan, pos)
        B.fmm_evaluate(plan, q, *out)
    for _ in range(warmup):
        g.replay()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record()
    for _ in range(steps):
        g.replay()
    t1.record()
    torch.cuda.synchronize()
    same = all(torch.equal(o, e) for o, e in zip(out, eager))
    st = B.fmm_check(plan)
    B.fmm_destroy(plan)
    return {"ms": t0.elapsed_time(t1) / steps, "value": n / (t0.elapsed_time(t1) / steps / 1e3),
            "equals_eager_bitwise": bool(same), "status": st}


def m2l_source_hash(variant):
    import hashlib
    h = hashlib.sha256()
    for f in VARIANTS[variant][3]:
        h.update(open(os.path.join(HERE, f), "rb").read())
    return h.hexdigest()


def m2l_traffic(variant):
    """HBM bytes per M2L kernel launch from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy's
    reading), or None when the summary is missing or was taken on different
    kernel source."""
    path = os.path.join(HERE, traffic_summary(variant))
    if not os.path.exists(path):
        return None
    src_hash, traffic = None, None
    for line in open(path):
        if line.startswith("source sha256:"):
            src_hash = line.split()[2]  # "source sha256: <hash>  (<files>)"
        if line.startswith("traffic_bytes_per_launch"):
            traffic = float(line.split()[-1])
    return traffic if src_hash == m2l_source_hash(variant) else None


def timed_steps(B, torch, pos, q, cfg, ws, steps, warmup, stream, breakdown_steps=3, schedule=None):
    """One plan (tree and translation operators), then warmup + steps of
    (fmm_replan + fmm_evaluate): the tree is rebuilt for the positions every
    step, the operator tables (a function of p and the M2L form only) are
    kept.  Returns ms/step, per-step HIP-event statistics, outputs of the last
    step, the M2L kernel durations over the timed steps (HIP events on the
    launch stream around that pass only), the per-pass durations of
    breakdown_steps further, untimed steps with every pass recorded, the
    status, the work counts, and the time of one fmm_plan with the operator
    generation."""
    n = q.numel()
    phi = torch.empty(n, dtype=torch.float64, device=pos.device)
    force = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    energy = torch.empty(1, dtype=torch.float64, device=pos.device)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    plan = B.fmm_plan(cfg, n, pos, ws, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    plan_ms = e0.elapsed_time(e1)
    if schedule:
        from paper_2209_13121_amd import autotune as T
        T.apply_schedule(plan, schedule)
    for _ in range(warmup):
        B.fmm_replan(plan, pos, stream)
        B.fmm_evaluate(plan, q, phi, force, energy, stream)
    torch.cuda.synchronize()
    B.fmm_profile_enable(plan, True, phases=["m2l"])
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record(stream)
    for i in range(steps):
        B.fmm_replan(plan, pos, stream)
        B.fmm_evaluate(plan, q, phi, force, energy, stream)
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    per_step = sorted(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
    step_stats = {"median_ms": per_step[steps // 2] if steps % 2 else
                  0.5 * (per_step[steps // 2 - 1] + per_step[steps // 2]),
                  "min_ms": per_step[0]}
    m2l = B.fmm_profile_read(plan)["m2l"]
    st = B.fmm_check(plan)
    work = B.fmm_plan_work(plan)
    B.fmm_profile_enable(plan, True)
    for _ in range(breakdown_steps):
        B.fmm_replan(plan, pos, stream)
        B.fmm_evaluate(plan, q, phi, force, energy, stream)
    torch.cuda.synchronize()
    phases = {k: [t / breakdown_steps, c / breakdown_steps]
              for k, (t, c) in B.fmm_profile_read(plan).items()}
    B.fmm_destroy(plan)
    return ms, step_stats, phi, force, energy, m2l, phases, st, work, plan_ms


def p2p_evidence(B, torch, pos, q, stream, depth=4, reps=3):
    """The near-field pass at a leaf occupancy where it carries real work: the
    same charges on a depth-4 tree (256 per leaf on average).  Returns, per
    precision, the P2P pass time (k_near, HIP events on the launch stream),
    the ordered pair count of the plan and the rate at 19 flop per pair."""
    n = q.numel()
    phi = torch.empty(n, dtype=torch.float64, device=pos.device)
    force = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    out = {}
    for prec, peak in (("MIXED", 157.3), ("FP64", 78.6)):
        cfg = B.make_config(p=8, depth=depth, precision=getattr(B, "FMM_PREC_" + prec))
        ws = torch.empty(B.fmm_workspace_size(cfg, n), dtype=torch.uint8, device=pos.device)
        t = c = 0.0
        for r in range(reps + 1):
            p = B.fmm_plan(cfg, n, pos, ws, stream)
            B.fmm_profile_enable(p, True, phases=["p2p"])
            B.fmm_evaluate(p, q, phi, force, None, stream)
            torch.cuda.synchronize()
            if r:  # the first is a warm-up
                tt, cc = B.fmm_profile_read(p)["p2p"]
                t += tt
                c += cc
            pairs = B.fmm_plan_work(p)[1]
            B.fmm_destroy(p)
        del ws
        ms = t / c
        tf = 19.0 * pairs / (ms / 1e3) / 1e12
        out[prec.lower()] = {"depth": depth, "pairs": pairs, "avg_ms": ms, "tflops": tf,
                             "vector_peak_tflops": peak, "frac": tf / peak}
    return out


def adaptive_bench(B, torch, args, stream):
    """The adaptive-tree workload (10^6 three-site clusters, leaves of at most
    64 sites, p = 10): plan + evaluate timed like the headline, mixed (FP16
    M2L, the library default) and FP64; accuracy of mixed against FP64 and of
    both against the exact sum on sampled sites; the M2L kernel's rate from the
    tree's own count of non-empty M2L pairs."""
    import numpy as np
    import oracle
    from paper_2209_13121_amd import workloads as W
    wl = W.CLUSTERS
    pos_np, q_np = wl.make()
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    res = {}
    for name, prec, kind, dtype, nprod, kernel in (
            ("mixed_f16x2", "MIXED", "F16X2", "f16", 3, "k_m2l_bf<10,2,f16>"),
            ("fp64", "FP64", "AUTO", "f64", 1, "k_m2l<10,double>")):
        cfg = B.make_config(p=wl.p, depth=wl.max_depth, precision=getattr(B, "FMM_PREC_" + prec),
                            m2l_kind=getattr(B, "FMM_M2L_" + kind), side=0.0, leaf_max=wl.leaf_max)
        nbytes = B.fmm_workspace_size(cfg, wl.n)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        print(f"[bench] adaptive {name}: workspace {nbytes / 2**20:.0f} MiB", file=sys.stderr, flush=True)
        ms, step_stats, phi, force, energy, m2l, phases, st, work, plan_ms = timed_steps(
            B, torch, pos, q, cfg, ws, max(5, args.steps // 2), args.warmup, stream)
        p = B.fmm_plan(cfg, wl.n, pos, ws, stream)
        stats = B.fmm_plan_tree_stats(p)
        B.fmm_destroy(p)
        t, c = m2l
        avg = t / c
        flops = 2.0 * (wl.p + 1) ** 4 * stats["m2l_pairs"]
        peak = PEAK_TFLOPS[dtype]
        res[name] = {"value": wl.n / (ms / 1e3), "ms_per_step": ms, "step_events_ms": step_stats,
                     "status": st, "first_plan_ms": plan_ms,
                     "phases_ms_per_step": {k: v[0] for k, v in phases.items()},
                     "m2l": {"kernel": kernel, "avg_launch_ms": avg, "flops_per_launch": flops,
                             "achieved": flops / (avg / 1e3) / 1e12, "peak": peak,
                             "frac": flops / (avg / 1e3) / 1e12 / peak,
                             "piece_products": nprod,
                             "piece_product_tflops": nprod * flops / (avg / 1e3) / 1e12},
                     "phi": phi.cpu().numpy(), "force": force.cpu().numpy(),
                     "energy": float(energy.cpu()[0])}
        print(f"[bench] adaptive {name}: {ms:.3f} ms/step, status {st}", file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
    m, f = res["mixed_f16x2"], res["fp64"]
    rng = np.random.default_rng(7)
    idx = rng.choice(wl.n, 256, replace=False)
    phi_d, force_d, _ = oracle.direct(pos_np, q_np, targets=idx)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    acc = {"rel_energy_err_vs_fp64_gpu": abs(m["energy"] - f["energy"]) / abs(f["energy"]),
           "rel_rms_force_err_vs_fp64_gpu": rel(m["force"], f["force"]),
           "rel_phi_err_vs_fp64_gpu": rel(m["phi"], f["phi"]),
           "rel_phi_err_vs_direct_256_sampled": {"mixed": rel(m["phi"][idx], phi_d),
                                                  "fp64": rel(f["phi"][idx], phi_d)},
           "rel_force_err_vs_direct_256_sampled": {"mixed": rel(m["force"][idx], force_d),
                                                    "fp64": rel(f["force"][idx], force_d)}}
    acc["gate_1e-6_met"] = bool(acc["rel_energy_err_vs_fp64_gpu"] <= 1e-6 and
                                acc["rel_rms_force_err_vs_fp64_gpu"] <= 1e-5)
    for r in res.values():
        for k in ("phi", "force", "energy"):
            r.pop(k)
    out = {"workload": wl.name, "n": wl.n, "leaf_max": wl.leaf_max, "depth_cap": wl.max_depth,
           "p": wl.p, "seed": wl.seed, "metric": "particles/s per FMM evaluation (tree build + evaluate)",
           "value": m["value"], "ms_per_step": m["ms_per_step"], "tree": stats, "accuracy": acc,
           "variants": res}
    if not args.no_cpu_baseline:
        sample = W.molecular_clusters(300_000, wl.seed)[:2]
        t0 = time.perf_counter()
        oracle.fmm_adaptive(sample[0], sample[1], wl.leaf_max, wl.max_depth, wl.p, side=0.0)
        dt = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {"value": len(sample[1]) / dt, "unit": "particles/s", "cores": threads,
                               "kind": "oracle",
                               "sample": f"CPU FP64 oracle adaptive FMM on 3e5 clusters (9e5 sites) of the "
                                         f"same recipe, leaf_max {wl.leaf_max}, p {wl.p}; {dt:.1f} s wall"}
    return out


def batch_bench(B, torch, args, stream):
    """The batch of 256 independent systems (10^3 .. 2^16 +-1 charges each,
    4.04e6 in all, p = 6): the autotuner picks the M2L form and the leaf
    capacity under the gate; then plan + evaluate of the whole batch is timed
    like the headline (one launch per pass for all systems), and the
    evaluation alone as one hipGraph replay."""
    import numpy as np
    import oracle
    from paper_2209_13121_amd import autotune as T
    from paper_2209_13121_amd import workloads as W
    wl = W.BATCH
    pos_np, q_np, counts = wl.make()
    n = len(q_np)
    grid = 1 << wl.batch_level
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    common = dict(lo=(0.0, 0.0, 0.0), side=float(grid), batch_level=wl.batch_level)
    print("[bench] batch: autotune", file=sys.stderr, flush=True)
    trees = [{"depth": wl.max_depth, "leaf_max": lm} for lm in (32, 64, 128)]
    best, table = T.tune(pos, q, wl.p, trees, reps=3, stream=stream, **common)
    tuned = ({"leaf_max": best.tree["leaf_max"], "m2l_kind": best.kind, "schedule": best.schedule}
             if best else None)
    kind = best.kind if best else "F16X2"
    leaf = best.tree["leaf_max"] if best else wl.leaf_max
    sched = best.schedule if best else {}
    res = {}
    for name, prec, mk in (("mixed", "MIXED", kind), ("fp64", "FP64", "AUTO")):
        cfg = B.make_config(p=wl.p, depth=wl.max_depth, precision=getattr(B, "FMM_PREC_" + prec),
                            m2l_kind=getattr(B, "FMM_M2L_" + mk), leaf_max=leaf, **common)
        ws = torch.empty(B.fmm_workspace_size(cfg, n), dtype=torch.uint8, device=dev)
        # the tuned schedule is the mixed form's; FP64 runs the default one
        sc = sched if name == "mixed" else {}
        ms, step_stats, phi, force, energy, m2l, phases, st, work, plan_ms = timed_steps(
            B, torch, pos, q, cfg, ws, max(5, args.steps // 2), args.warmup, stream, schedule=sc)
        entry = {"value": n / (ms / 1e3), "ms_per_step": ms, "step_events_ms": step_stats, "status": st,
                 "schedule": sc,
                 "first_plan_ms": plan_ms,
                 "phases_ms_per_step": {k: v[0] for k, v in phases.items()},
                 "m2l_avg_launch_ms": m2l[0] / m2l[1]}
        if name == "mixed":
            # the evaluation alone, captured once and replayed as one graph launch
            plan = B.fmm_plan(cfg, n, pos, ws, stream)
            T.apply_schedule(plan, sc)
            ph = torch.empty(n, dtype=torch.float64, device=dev)
            fo = torch.empty((n, 3), dtype=torch.float64, device=dev)
            en = torch.empty(1, dtype=torch.float64, device=dev)
            side_s = torch.cuda.Stream()
            side_s.wait_stream(stream)
            with torch.cuda.stream(side_s):
                B.fmm_evaluate(plan, q, ph, fo, en)
            stream.wait_stream(side_s)
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g):
                B.fmm_evaluate(plan, q, ph, fo, en)
            g.replay()
            torch.cuda.synchronize()
            reps = max(5, args.steps // 2)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                g.replay()
            e1.record()
            torch.cuda.synchronize()
            gms = e0.elapsed_time(e1) / reps
            entry["graph_evaluate"] = {"ms": gms, "value": n / (gms / 1e3),
                                       "equals_eager_bitwise": bool(torch.equal(ph, phi))}
            B.fmm_destroy(plan)
            del g
        res[name] = dict(entry, phi=phi.cpu().numpy(), force=force.cpu().numpy(),
                         energy=float(energy.cpu()[0]), work=work)
        print(f"[bench] batch {name}: {ms:.3f} ms/step, status {st}", file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()
    m, f = res["mixed"], res["fp64"]
    acc = {"rel_energy_err_vs_fp64_gpu": abs(m["energy"] - f["energy"]) / abs(f["energy"]),
           "rel_rms_force_err_vs_fp64_gpu": float(np.linalg.norm(m["force"] - f["force"]) /
                                                  np.linalg.norm(f["force"]))}
    # FP64 against the oracle of three systems alone (smallest, middle, largest)
    starts = np.concatenate([[0], np.cumsum(counts)])
    errs = {}
    for k in (int(np.argmin(counts)), len(counts) // 2, int(np.argmax(counts))):
        sl = slice(starts[k], starts[k + 1])
        cell = (k % grid, (k // grid) % grid, k // (grid * grid))
        ph, fo, _, _ = oracle.fmm_adaptive(pos_np[sl], q_np[sl], leaf, wl.max_depth - wl.batch_level,
                                           wl.p, lo=cell, side=1.0)
        errs[str(k)] = float(np.linalg.norm(f["phi"][sl] - ph) / np.linalg.norm(ph))
    acc["fp64_rel_phi_err_vs_oracle_systems"] = errs
    acc["gate_1e-6_met"] = bool(acc["rel_energy_err_vs_fp64_gpu"] <= 1e-6 and
                                acc["rel_rms_force_err_vs_fp64_gpu"] <= 1e-5)
    for r in res.values():
        for k in ("phi", "force", "energy"):
            r.pop(k)
    out = {"workload": wl.name, "n": n, "systems": wl.n_systems, "n_min": int(counts.min()),
           "n_max": int(counts.max()), "p": wl.p, "depth_cap": wl.max_depth, "batch_level": wl.batch_level,
           "seed": wl.seed, "metric": "aggregate particles/s per batch evaluation (tree build + evaluate)",
           "value": m["value"], "ms_per_step": m["ms_per_step"], "tuned": tuned,
           "autotune": [{"leaf_max": r.tree["leaf_max"], "m2l_kind": r.kind, "schedule": r.schedule,
                         "ms": r.ms, "energy_err": r.energy_err, "force_err": r.force_err} for r in table],
           "accuracy": acc, "variants": res}
    if not args.no_cpu_baseline:
        t0 = time.perf_counter()
        done = 0
        for k in range(160):  # the first 160 systems, each alone
            sl = slice(starts[k], starts[k + 1])
            cell = (k % grid, (k // grid) % grid, k // (grid * grid))
            oracle.fmm_adaptive(pos_np[sl], q_np[sl], leaf, wl.max_depth - wl.batch_level, wl.p,
                                lo=cell, side=1.0)
            done += counts[k]
        dt = time.perf_counter() - t0
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = {"value": done / dt, "unit": "particles/s", "cores": threads, "kind": "oracle",
                               "sample": f"CPU FP64 oracle adaptive FMM of the first 160 systems "
                                         f"({int(done)} charges), one after another; {dt:.1f} s wall"}
    return out


def cpu_baseline(pos, q, wl, nboxes, reps=3):
    """The oracle as it stands, timed on this host: the FP64 FMM evaluated at
    the particles of nboxes of the 8 level-1 boxes (full upward pass, M2L and
    L2L for the ancestors of those particles' leaves), median of reps runs;
    and the exact O(N^2) sum at 4,096 targets, scaled to particles/s
    (extrapolated: a full direct sum would take N / 4096 times as long)."""
    import numpy as np
    import oracle
    half = (pos >= 0.5).astype(int)
    box = half[:, 0] * 4 + half[:, 1] * 2 + half[:, 2]
    targets = np.nonzero(box < nboxes)[0]
    times = []
    for _ in range(reps):
        t0 = time.perf_counter()
        oracle.fmm(pos, q, wl.depth, wl.p, targets=targets)
        times.append(time.perf_counter() - t0)
    dt = sorted(times)[len(times) // 2]
    dsub = np.arange(0, len(q), len(q) // 4096)[:4096]
    t0 = time.perf_counter()
    oracle.direct(pos, q, targets=dsub)
    ddt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model, ncpu = host_cpu()
    return {"value": len(targets) / dt, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": f"CPU FP64 oracle FMM (same tree, p) at the {len(targets)} particles of "
                      f"{nboxes} of the 8 level-1 boxes, full upward pass; median of {reps}: "
                      f"{dt:.1f} s",
            "host": {"cpu_model": model, "nproc": ncpu, "omp_threads": threads},
            "direct_sum": {"value": len(dsub) / ddt, "unit": "particles/s",
                           "sample": f"O(N^2) sum at {len(dsub)} of {len(q)} targets, {ddt:.1f} s; "
                                     f"a full sum extrapolates to {ddt * len(q) / len(dsub):.0f} s"}}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "this build has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    from paper_2209_13121_amd import binding as B
    from paper_2209_13121_amd import workloads as W

    if args.adaptive_only:
        B.load()
        print(json.dumps(adaptive_bench(B, torch, args, torch.cuda.current_stream())), flush=True)
        return
    if args.batch_only:
        B.load()
        print(json.dumps(batch_bench(B, torch, args, torch.cuda.current_stream())), flush=True)
        return
    wl = W.HEADLINE
    pos_np, q_np = wl.make()
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    stream = torch.cuda.current_stream()
    B.load()
    if args.p2p_only:
        print(json.dumps({"p2p_depth4": p2p_evidence(B, torch, pos, q, stream)}), flush=True)
        return

    results = {}
    for name, (prec, kind, *_rest) in VARIANTS.items():
        if args.only and name != args.only:
            continue
        cfg = B.make_config(p=wl.p, depth=wl.depth, precision=getattr(B, "FMM_PREC_" + prec),
                            m2l_kind=getattr(B, "FMM_M2L_" + kind))
        nbytes = B.fmm_workspace_size(cfg, wl.n)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        print(f"[bench] {name}: workspace {nbytes / 2**20:.0f} MiB", file=sys.stderr, flush=True)
        ms, step_stats, phi, force, energy, m2l, phases, st, work, plan_ms = timed_steps(
            B, torch, pos, q, cfg, ws, args.steps, args.warmup, stream)
        results[name] = dict(ms=ms, step_stats=step_stats, phi=phi.cpu().numpy(),
                             force=force.cpu().numpy(),
                             energy=float(energy.cpu()[0]), m2l=m2l, phases=phases, status=st,
                             work=work, plan_ms=plan_ms)
        if name == HEADLINE:
            results[name]["graph_step"] = graph_step(B, torch, pos, q, cfg, ws, args.steps, args.warmup)
        print(f"[bench] {name}: {ms:.3f} ms/step, status {st}", file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()

    if args.only:
        r = results[args.only]
        print(json.dumps({"only": args.only, "ms_per_step": r["ms"],
                          "value": wl.n / (r["ms"] / 1e3), "status": r["status"],
                          "phases_ms_per_step": {k: v[0] for k, v in r["phases"].items()}}),
              flush=True)
        return
    golden_path = os.path.join(HERE, "tests", "golden", "headline_oracle.json")
    e_ref = json.load(open(golden_path))[wl.name]["energy"] if os.path.exists(golden_path) else None
    f64 = results["fp64"]

    def erel(e):
        return abs(e - e_ref) / abs(e_ref) if e_ref is not None else None

    nc = (wl.p + 1) ** 2
    m2l_pairs, p2p_pairs = f64["work"]
    m2l_flops = 2.0 * nc * nc * m2l_pairs  # algorithmic, non-empty box pairs

    def m2l_rate(name):
        """Average M2L launch (ms) and the kernel's rate in the method's own
        work (2 ncoef^2 flop per non-empty box pair, counted once) against the
        dense matrix peak of the dtype its matrix cores run; the rate of the
        piece products the split forms execute is a separate figure."""
        _, _, kernel, _, dtype, nprod = VARIANTS[name]
        t, c = results[name]["m2l"]
        avg_ms = t / c
        ach = m2l_flops / (avg_ms / 1e3) / 1e12
        return {"kernel": kernel, "avg_launch_ms": avg_ms, "flops_per_launch": m2l_flops,
                "achieved": ach, "peak": PEAK_TFLOPS[dtype], "frac": ach / PEAK_TFLOPS[dtype],
                "piece_products": nprod, "piece_product_tflops": nprod * ach}

    variants = {}
    for name, r in results.items():
        variants[name] = {
            "value": wl.n / (r["ms"] / 1e3), "ms_per_step": r["ms"], "status": r["status"],
            "step_events_ms": r["step_stats"],
            "rel_energy_err_vs_oracle": erel(r["energy"]),
            "rel_rms_force_err_vs_fp64_gpu": float(
                np.linalg.norm(r["force"] - f64["force"]) / np.linalg.norm(f64["force"])),
            "rel_phi_err_vs_fp64_gpu": float(
                np.linalg.norm(r["phi"] - f64["phi"]) / np.linalg.norm(f64["phi"])),
            "phases_ms_per_step": {k: v[0] for k, v in r["phases"].items()},
            "m2l": m2l_rate(name),
            "first_plan_ms": r["plan_ms"],
        }
        if "graph_step" in r:
            variants[name]["graph_step"] = r["graph_step"]
    golden = load_golden(wl)
    acc = {name: accuracy_vs_oracle(r, golden) for name, r in results.items()}
    for name in variants:
        variants[name].update(acc[name])
    hl = variants[HEADLINE]
    gate = bool(hl["rel_energy_err_vs_oracle"] is not None and hl["rel_energy_err_vs_oracle"] <= 1e-6
                and hl["rel_rms_force_err_vs_oracle_sampled"] is not None
                and hl["rel_rms_force_err_vs_oracle_sampled"] <= 1e-5
                and hl["rel_rms_force_err_vs_fp64_gpu"] <= 1e-5)
    rate = hl["m2l"]
    roofline = {"bound": "mfma", "kernel": rate["kernel"], "achieved": rate["achieved"],
                "peak": rate["peak"], "unit": "TFLOP/s", "frac": rate["frac"],
                "traffic": m2l_traffic(HEADLINE), "flops_per_launch": rate["flops_per_launch"],
                "m2l_pairs": m2l_pairs, "avg_launch_ms": rate["avg_launch_ms"],
                "piece_products": rate["piece_products"],
                "piece_product_tflops": rate["piece_product_tflops"]}

    out = {
        "metric": METRIC,
        "value": hl["value"],
        "unit": "particles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hl["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": VARIANTS[HEADLINE][4] + "/f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "depth": wl.depth, "p": wl.p, "seed": wl.seed,
                   "variant": HEADLINE,
                   "precision": "mixed (FP32 P2M/L2P/P2P, M2L on " +
                                {"f16": "scaled split-FP16 MFMA, 2 pieces",
                                 "bf16": "split-BF16 MFMA, 3 pieces",
                                 "f32": "FP32 MFMA"}[VARIANTS[HEADLINE][4]] +
                                ", FP64 M2M/L2L/energy)",
                   "step": "fmm_replan (tree build) + fmm_evaluate; operators from the first fmm_plan"},
        "roofline": roofline,
    }
    detail = {"variants": variants, "p2p_pairs": p2p_pairs}
    print("[bench] p2p at depth 4", file=sys.stderr, flush=True)
    detail["p2p_depth4"] = p2p_evidence(B, torch, pos, q, stream)
    print("[bench] small workload against the direct sum", file=sys.stderr, flush=True)
    detail["small"] = small_workload(B, torch)
    if not args.no_adaptive:
        del pos, q
        torch.cuda.empty_cache()
        detail["adaptive"] = adaptive_bench(B, torch, args, stream)
        torch.cuda.empty_cache()
        detail["batch"] = batch_bench(B, torch, args, stream)
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pos_np, q_np, wl, args.cpu_sample_boxes)
    # The full record goes to stderr; the JSON line on stdout keeps the contract
    # keys, a compact summary of every workload, and the headline accuracy last.
    print("[bench-detail] " + json.dumps(detail), file=sys.stderr, flush=True)
    out["variants"] = {k: {"ms": v["ms_per_step"], "m2l_ms": v["m2l"]["avg_launch_ms"],
                           "m2l_frac": v["m2l"]["frac"], "dE": v["rel_energy_err_vs_oracle"],
                           "dF": v["rel_rms_force_err_vs_oracle_sampled"]}
                       for k, v in variants.items()}
    if "graph_step" in hl:
        out["variants"][HEADLINE]["graph_step_ms"] = hl["graph_step"]["ms"]
    out["p2p_depth4_frac"] = {k: v["frac"] for k, v in detail["p2p_depth4"].items()}
    out["small"] = detail["small"]
    for key in ("adaptive", "batch"):
        if key in detail:
            d = detail[key]
            out[key] = {"workload": d["workload"], "value": d["value"], "ms": d["ms_per_step"],
                        "fp64_ms": d["variants"]["fp64"]["ms_per_step"],
                        "dE_vs_fp64": d["accuracy"]["rel_energy_err_vs_fp64_gpu"],
                        "dF_vs_fp64": d["accuracy"]["rel_rms_force_err_vs_fp64_gpu"],
                        "gate_met": d["accuracy"]["gate_1e-6_met"]}
            if "cpu_baseline" in d:
                out[key]["cpu_particles_per_s"] = d["cpu_baseline"]["value"]
            if key == "batch":
                out[key]["tuned"] = d["tuned"]
                out[key]["graph_evaluate_ms"] = d["variants"]["mixed"]["graph_evaluate"]["ms"]
    out["accuracy"] = {
        "rel_energy_err_vs_oracle": hl["rel_energy_err_vs_oracle"],
        "rel_rms_force_err_vs_oracle_sampled": hl["rel_rms_force_err_vs_oracle_sampled"],
        "rel_phi_err_vs_oracle_sampled": hl["rel_phi_err_vs_oracle_sampled"],
        "rel_rms_force_err_vs_fp64_gpu": hl["rel_rms_force_err_vs_fp64_gpu"],
        "fp64_rel_energy_err_vs_oracle": variants["fp64"]["rel_energy_err_vs_oracle"],
        "rel_phi_err_vs_direct_32k": hl["rel_phi_err_vs_direct_32k"],
        "rel_force_err_vs_direct_32k": hl["rel_force_err_vs_direct_32k"],
        "gate_1e-6_met": gate}
    print(json.dumps(out), flush=True)


def load_golden(wl):
    """Stored oracle values of the headline workload (tests/golden, written by
    make_golden.py from the oracle only): energy, sampled potentials and
    forces, exact sums at 32,768 particles."""
    import numpy as np
    g = {}
    path = os.path.join(HERE, "tests", "golden", "headline_oracle.json")
    if os.path.exists(path):
        g.update(json.load(open(path))[wl.name])
    path = os.path.join(HERE, "tests", "golden", "headline_direct_32k.npz")
    if os.path.exists(path):
        with np.load(path, allow_pickle=False) as z:
            g["direct"] = {k: z[k] for k in ("index", "phi", "force")}
    return g


def accuracy_vs_oracle(r, golden):
    import numpy as np

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    out = {"rel_energy_err_vs_oracle": None, "rel_rms_force_err_vs_oracle_sampled": None,
           "rel_phi_err_vs_oracle_sampled": None, "rel_phi_err_vs_direct_32k": None,
           "rel_force_err_vs_direct_32k": None}
    if "energy" in golden:
        out["rel_energy_err_vs_oracle"] = abs(r["energy"] - golden["energy"]) / abs(golden["energy"])
    if "sample_index" in golden:
        s = np.array(golden["sample_index"])
        out["rel_rms_force_err_vs_oracle_sampled"] = rel(r["force"][s], np.array(golden["sample_force"]))
        out["rel_phi_err_vs_oracle_sampled"] = rel(r["phi"][s], np.array(golden["sample_phi"]))
    if "direct" in golden:
        d = golden["direct"]
        out["rel_phi_err_vs_direct_32k"] = rel(r["phi"][d["index"]], d["phi"])
        out["rel_force_err_vs_direct_32k"] = rel(r["force"][d["index"]], d["force"])
    return out


def small_workload(B, torch):
    """The 4,096-charge workload (depth 3, p = 4, FP64): the library's result
    against the exact O(N^2) sums and against the oracle FMM."""
    import numpy as np
    import oracle
    from paper_2209_13121_amd import workloads as W
    wl = W.SMALL
    pos_np, q_np = wl.make()
    dev = torch.device("cuda:0")
    f = B.FMM(torch.from_numpy(pos_np).to(dev), p=wl.p, depth=wl.depth)
    phi, force, e = f.evaluate(torch.from_numpy(q_np).to(dev))
    st = f.check()
    f.close()
    phi, force, e = phi.cpu().numpy(), force.cpu().numpy(), float(e.cpu()[0])
    phi_d, force_d, e_d = oracle.direct(pos_np, q_np)
    phi_o, force_o, e_o = oracle.fmm(pos_np, q_np, wl.depth, wl.p)

    def rel(a, b):
        return float(np.linalg.norm(a - b) / np.linalg.norm(b))
    return {"workload": wl.name, "status": st,
            "vs_direct": {"dE": abs(e - e_d) / abs(e_d), "dF": rel(force, force_d), "dphi": rel(phi, phi_d)},
            "vs_oracle": {"dE": abs(e - e_o) / abs(e_o), "dF": rel(force, force_o), "dphi": rel(phi, phi_o)}}


def host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count()


if __name__ == "__main__":
    main()
