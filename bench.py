"""Benchmark: FMM throughput on one MI355X (particles per second per evaluation).

Workload: 2^20 charges uniform in the unit cube, Gaussian charges shifted to
net zero (seed 1002), uniform octree of depth 6, expansion order p = 8.  One
step = fmm_plan (tree build for the positions) + fmm_evaluate (all passes,
potentials, forces and energy) on device-resident inputs.  The headline value
is the mixed-precision path; the FP64 path is timed the same way and reported
beside it, with both energies compared to the stored FP64 oracle energy.

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
M2L_SOURCES = ["paper_2209_13121_amd/csrc/m2l.hip", "paper_2209_13121_amd/csrc/fmm_internal.h"]
TRAFFIC_SUMMARY = "profiles/k_m2l_mixed_uniform-gauss-n1048576-depth6-p8_hbm_counters.txt"
PEAK_TFLOPS = {"f32": 157.3, "f64": 78.6}  # MI355X dense matrix peaks


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-boxes", type=int, default=1,
                    help="level-1 boxes (1/8 of the domain each) whose particles the oracle evaluates")
    ap.add_argument("--only", choices=["mixed", "fp64"], default=None,
                    help="time one precision only (profiling runs)")
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


def m2l_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in M2L_SOURCES:
        h.update(open(os.path.join(HERE, f), "rb").read())
    return h.hexdigest()


def m2l_traffic():
    """HBM bytes per k_m2l launch from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by a plain copy's reading), or
    None when the summary is missing or was taken on different kernel source."""
    path = os.path.join(HERE, TRAFFIC_SUMMARY)
    if not os.path.exists(path):
        return None
    src_hash, traffic = None, None
    for line in open(path):
        if line.startswith("source sha256:"):
            src_hash = line.split()[-1]
        if line.startswith("traffic_bytes_per_launch"):
            traffic = float(line.split()[-1])
    return traffic if src_hash == m2l_source_hash() else None


def timed_steps(B, torch, pos, q, cfg, ws, steps, warmup, stream):
    """Run warmup + steps of (plan + evaluate); returns ms/step, outputs of the
    last step and the per-phase kernel durations over the timed steps."""
    n = q.numel()
    phi = torch.empty(n, dtype=torch.float64, device=pos.device)
    force = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
    energy = torch.empty(1, dtype=torch.float64, device=pos.device)
    plans = []
    for _ in range(warmup):
        p = B.fmm_plan(cfg, n, pos, ws, stream)
        B.fmm_evaluate(p, q, phi, force, energy, stream)
        plans.append(p)
    torch.cuda.synchronize()
    for p in plans:
        B.fmm_destroy(p)
    plans = []
    t0 = time.perf_counter()
    for _ in range(steps):
        p = B.fmm_plan(cfg, n, pos, ws, stream)
        B.fmm_profile_enable(p, True)
        B.fmm_evaluate(p, q, phi, force, energy, stream)
        plans.append(p)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    # kernel durations recorded with HIP events on the launch stream
    phases = {}
    for p in plans:
        for k, (t, c) in B.fmm_profile_read(p).items():
            a = phases.setdefault(k, [0.0, 0])
            a[0] += t
            a[1] += c
    st = B.fmm_check(plans[-1])
    work = B.fmm_plan_work(plans[-1])
    for p in plans:
        B.fmm_destroy(p)
    return ms, phi, force, energy, phases, st, work


def cpu_baseline(pos, q, wl, nboxes):
    import numpy as np
    import oracle
    half = (pos >= 0.5).astype(int)
    box = half[:, 0] * 4 + half[:, 1] * 2 + half[:, 2]
    targets = np.nonzero(box < nboxes)[0]
    t0 = time.perf_counter()
    oracle.fmm(pos, q, wl.depth, wl.p, targets=targets)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": len(targets) / dt, "unit": "particles/s", "cores": threads, "kind": "oracle",
            "sample": f"CPU FP64 oracle FMM (same tree, p) evaluated at the {len(targets)} particles "
                      f"of {nboxes} of the 8 level-1 boxes, full upward pass included; "
                      f"{dt:.1f} s wall"}


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

    wl = W.HEADLINE
    pos_np, q_np = wl.make()
    dev = torch.device("cuda:0")
    pos = torch.from_numpy(pos_np).to(dev)
    q = torch.from_numpy(q_np).to(dev)
    stream = torch.cuda.current_stream()
    B.load()

    results = {}
    for name, prec in (("mixed", B.FMM_PREC_MIXED), ("fp64", B.FMM_PREC_FP64)):
        if args.only and name != args.only:
            continue
        cfg = B.make_config(p=wl.p, depth=wl.depth, precision=prec)
        nbytes = B.fmm_workspace_size(cfg, wl.n)
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        print(f"[bench] {name}: workspace {nbytes / 2**20:.0f} MiB", file=sys.stderr, flush=True)
        ms, phi, force, energy, phases, st, work = timed_steps(
            B, torch, pos, q, cfg, ws, args.steps, args.warmup, stream)
        results[name] = dict(ms=ms, phi=phi.cpu().numpy(), force=force.cpu().numpy(),
                             energy=float(energy.cpu()[0]), phases=phases, status=st, work=work)
        print(f"[bench] {name}: {ms:.3f} ms/step, status {st}", file=sys.stderr, flush=True)
        del ws
        torch.cuda.empty_cache()

    if args.only:
        r = results[args.only]
        print(json.dumps({"only": args.only, "ms_per_step": r["ms"],
                          "value": wl.n / (r["ms"] / 1e3), "status": r["status"],
                          "phases_ms_per_step": {k: v[0] / args.steps for k, v in r["phases"].items()}}),
              flush=True)
        return
    golden_path = os.path.join(HERE, "tests", "golden", "headline_oracle.json")
    e_ref = json.load(open(golden_path))[wl.name]["energy"] if os.path.exists(golden_path) else None
    mx, f64 = results["mixed"], results["fp64"]

    def erel(e):
        return abs(e - e_ref) / abs(e_ref) if e_ref is not None else None

    acc = {
        "oracle_energy": e_ref,
        "mixed_rel_energy_err_vs_oracle": erel(mx["energy"]),
        "fp64_rel_energy_err_vs_oracle": erel(f64["energy"]),
        "mixed_rel_rms_force_err_vs_fp64_gpu": float(
            np.linalg.norm(mx["force"] - f64["force"]) / np.linalg.norm(f64["force"])),
        "mixed_rel_phi_err_vs_fp64_gpu": float(
            np.linalg.norm(mx["phi"] - f64["phi"]) / np.linalg.norm(f64["phi"])),
    }
    gate = acc["mixed_rel_energy_err_vs_oracle"] is not None and \
        acc["mixed_rel_energy_err_vs_oracle"] <= 1e-6
    acc["gate_1e-6_met"] = bool(gate)

    nc = (wl.p + 1) ** 2
    m2l_pairs, p2p_pairs = mx["work"]
    m2l_flops = 2.0 * nc * nc * m2l_pairs  # algorithmic, non-empty box pairs
    t_m2l, n_m2l = mx["phases"]["m2l"]
    avg_m2l_s = t_m2l / n_m2l / 1e3
    achieved = m2l_flops / avg_m2l_s / 1e12
    t64, n64 = f64["phases"]["m2l"]
    roofline = {"bound": "mfma", "kernel": "k_m2l<8,float>", "achieved": achieved,
                "peak": PEAK_TFLOPS["f32"], "unit": "TFLOP/s", "frac": achieved / PEAK_TFLOPS["f32"],
                "traffic": m2l_traffic(), "flops_per_launch": m2l_flops, "m2l_pairs": m2l_pairs,
                "avg_launch_ms": t_m2l / n_m2l,
                "fp64_kernel_achieved": m2l_flops / (t64 / n64 / 1e3) / 1e12,
                "fp64_kernel_frac": m2l_flops / (t64 / n64 / 1e3) / 1e12 / PEAK_TFLOPS["f64"]}

    out = {
        "metric": METRIC,
        "value": wl.n / (mx["ms"] / 1e3),
        "unit": "particles/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": mx["ms"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl.name, "n": wl.n, "depth": wl.depth, "p": wl.p, "seed": wl.seed,
                   "precision": "mixed (FP32 P2M/M2L-MFMA/L2P/P2P, FP64 M2M/L2L/energy)",
                   "step": "fmm_plan + fmm_evaluate"},
        "fp64": {"value": wl.n / (f64["ms"] / 1e3), "ms_per_step": f64["ms"]},
        "accuracy": acc,
        "phases_ms_per_step": {k: v[0] / args.steps for k, v in mx["phases"].items()},
        "fp64_phases_ms_per_step": {k: v[0] / args.steps for k, v in f64["phases"].items()},
        "p2p_pairs": p2p_pairs,
        "roofline": roofline,
        "status": {"mixed": mx["status"], "fp64": f64["status"]},
    }
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(pos_np, q_np, wl, args.cpu_sample_boxes)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
