"""Benchmark of the aggregated FP64 sub-grid hydro step on one MI355X.

Default workload: 4096 independent sub-grids of 8^3 cells (+3 ghost layers,
14^3 stored), 11 FP64 fields, the random smooth state (seeded), dx = 1/64,
dt from a dt = 0 pass at Courant number 0.4.  One timed step = one stage of
the step over the whole batch, issued as ONE hipGraph launch of the
aggregated kernel (inputs resident in HBM before the timed region).

Also measured, on the same GPU and inputs: the same kernel launched once per
sub-grid (4096 launches, the non-aggregated baseline), and the CPU oracle on
the host cores (cpu_baseline).  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "FP64 hydro cell-updates/s aggregated vs per-subgrid launch; %HBM roofline; p99 latency"
HBM_PEAK_GBS = 8000.0
GHOST = 3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_subgrid(n, nf):
    """Algorithmic HBM bytes of one sub-grid step.
    floor: the cells the face-centred stencil reads (interior + the six 3-deep
    face slabs) once, plus the interior written once.
    tile: the whole stored (n+6)^3 block read once, plus the interior written."""
    M = n + 2 * GHOST
    floor = (n ** 3 + 6 * GHOST * n ** 2 + n ** 3) * nf * 8
    tile = (M ** 3 + n ** 3) * nf * 8
    return floor, tile


def measured_traffic(version, workload):
    """HBM bytes per launch from the committed rocprofv3 counter record, or
    None when that record was taken on another build of the kernel."""
    path = os.path.join(ROOT, "paper_2210_06438_amd", "measured_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_version") != version or rec.get("workload") != workload:
        return None
    return int(rec["traffic_bytes_per_launch"])


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--n", type=int, default=8)
    ap.add_argument("--nfields", type=int, default=11)
    ap.add_argument("--each-reps", type=int, default=3,
                    help="timed repetitions of the one-launch-per-sub-grid baseline")
    ap.add_argument("--cpu-reps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="minimum wall time of the oracle measurement")
    ap.add_argument("--copy-reps", type=int, default=10,
                    help="timed repetitions of a plain device copy of the input buffer")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0,
                    help="oracle threads (0 = OMP_NUM_THREADS or all cores)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2210_06438_amd import hydroagg, workloads

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    hydroagg.lib()   # fail loudly if the HIP library is missing

    count, n, nf = args.count, args.n, args.nfields
    dx = 1.0 / 64
    log(f"generating {count} sub-grids n={n} F={nf}")
    t0 = time.time()
    U = workloads.random_smooth(count, n=n, nfields=nf, seed=2)
    log(f"generated in {time.time() - t0:.1f}s ({U.nbytes / 1e9:.2f} GB)")
    u_in = torch.from_numpy(U).to(dev)
    u_out = u_in.clone()
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    descs = hydroagg.subgrids(u_in, u_out)
    plan = hydroagg.Plan(descs)
    stream = torch.cuda.current_stream()

    plan.step(0.0, dx, amax, stream)
    torch.cuda.synchronize()
    dt = 0.4 * dx / float(amax.max())
    log(f"dt = {dt:.6e}; library {hydroagg.version()}")

    # ---- aggregated: one hipGraph launch per step -------------------------
    for _ in range(args.warmup):
        plan.graph(dt, dx, amax, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        plan.graph(dt, dx, amax, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    cells = count * n ** 3
    value = cells / (ms * 1e-3)
    log(f"aggregated: {ms * 1e3:.1f} us/step, {value / 1e9:.3f} G cell-updates/s")

    # ---- baseline: the same kernel, one launch per sub-grid ----------------
    each_ms = None
    if args.each_reps > 0:
        hydroagg.hydro_step_each(descs, dt, dx, amax, stream)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.each_reps):
            hydroagg.hydro_step_each(descs, dt, dx, amax, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        each_ms = e0.elapsed_time(e1) / args.each_reps
        log(f"per-sub-grid launches: {each_ms:.2f} ms/step")

    # ---- a plain device copy of the same buffer: measured bandwidth reference
    copy_gbs = None
    if args.copy_reps > 0:
        u_out.copy_(u_in)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.copy_reps):
            u_out.copy_(u_in)
        e1.record(stream)
        torch.cuda.synchronize()
        copy_ms = e0.elapsed_time(e1) / args.copy_reps
        copy_gbs = 2 * u_in.numel() * 8 / (copy_ms * 1e-3) / 1e9
        log(f"device copy of {u_in.numel() * 8 / 1e9:.2f} GB: {copy_ms * 1e3:.1f} us, {copy_gbs:.0f} GB/s")

    floor_b, tile_b = bytes_per_subgrid(n, nf)
    achieved = tile_b * count / (ms * 1e-3) / 1e9
    achieved_floor = floor_b * count / (ms * 1e-3) / 1e9
    version = hydroagg.version()
    workload_name = f"{count}x{n}^3 F={nf}"
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(version, workload_name),
        "kernel": (f"hydro_lds8_kernel<{nf}>" if n == 8 else f"hydro_table_kernel<{n},{nf}>"),
        "kernel_version": version,
        "algorithmic_bytes_per_launch": tile_b * count,
        "bytes_definition": "stored (n+6)^3 tile read once + interior n^3 written once, 8 B x F per cell",
        "achieved_floor_gbs": round(achieved_floor, 1),
        "floor_bytes_per_launch": floor_b * count,
        "measured_copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
    }

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS", "0") or 0) \
            or os.cpu_count() or 1
        log(f"cpu baseline: oracle on the full batch, {threads} threads, "
            f">= {args.cpu_seconds:.0f} s")
        times = []
        t_all = time.time()
        while len(times) < max(args.cpu_reps, 1) or time.time() - t_all < args.cpu_seconds:
            t0 = time.time()
            oracle.step(U, dt, dx, nthreads=threads)
            times.append(time.time() - t0)
        med = statistics.median(times)
        cpu = {"value": round(cells / med, 1), "unit": "cell-updates/s", "cores": threads,
               "kind": "oracle",
               "sample": f"the full {count}-sub-grid workload stepped {len(times)} times "
                         f"({sum(times):.1f} s wall, median {med:.3f} s per step), "
                         "OpenMP over sub-grids"}
        log(f"cpu baseline {cells / med / 1e6:.2f} M cell-updates/s")

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{count} sub-grids of {n}^3 (+3 ghost layers), {nf} FP64 fields, "
                        "random smooth state, one aggregated hipGraph launch per step",
            "subgrids": count, "n": n, "nfields": nf, "dx": dx, "cfl": 0.4,
        },
        "per_subgrid_launch": None if each_ms is None else {
            "value": round(cells / (each_ms * 1e-3), 1), "ms_per_step": round(each_ms, 4),
            "launches_per_step": count},
        "aggregation_speedup": None if each_ms is None else round(each_ms / ms, 2),
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
