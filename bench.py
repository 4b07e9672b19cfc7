"""Benchmark of the aggregated FP64 sub-grid hydro step on one MI355X.

Default workload: 4096 independent sub-grids of 8^3 cells (+3 ghost layers,
14^3 stored), 11 FP64 fields, the random smooth state (seeded), dx = 1/64,
dt from a dt = 0 pass at Courant number 0.4.  One timed step = one stage of
the step over the whole batch, issued as ONE hipGraph launch of the
aggregated kernel (inputs resident in HBM before the timed region), each
sub-grid's updated interior written to [F][n][n][n] (the stored (n+6)^3
output layout is timed beside it).

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
FP64_PEAK_TFLOPS = 78.6
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


def kernels_hash(version):
    """The "kernels <hash>" part of hydro_version(), or None."""
    parts = version.split()
    return parts[parts.index("kernels") + 1] if "kernels" in parts[:-1] else None


def counter_record(name, version, workload, kernel, path=None):
    """A committed rocprofv3 counter record (paper_2210_06438_amd/<name>),
    or None when it was taken on other kernels (their sources or flags
    differ), another workload or another kernel."""
    if path is None:
        path = os.path.join(ROOT, "paper_2210_06438_amd", name)
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    here = kernels_hash(version)
    if here is None or kernels_hash(rec.get("kernel_version", "")) != here:
        return None
    if rec.get("workload") != workload:
        return None
    if kernel.split("<")[0] not in rec.get("kernel", ""):
        return None
    return rec


def measured_traffic(version, workload, kernel, path=None):
    """HBM bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)."""
    rec = counter_record("measured_traffic.json", version, workload, kernel, path)
    return None if rec is None else int(rec["traffic_bytes_per_launch"])


def measured_fp64(version, workload, kernel, kernel_ms, path=None):
    """FP64 operations per launch (SQ_INSTS_VALU_*_F64) and the rate they
    give at the kernel duration measured in this run."""
    rec = counter_record("measured_fp64.json", version, workload, kernel, path)
    if rec is None:
        return None
    flop = float(rec["fp64_flop_per_launch"])
    tflops = flop / (kernel_ms * 1e-3) / 1e12
    return {"flop_per_launch": int(flop), "achieved_tflops": round(tflops, 2),
            "peak_tflops": FP64_PEAK_TFLOPS, "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
            "valu_insts_per_wave": round(float(rec["valu_insts_per_wave"]), 1)}


def uneven_leg(args, torch, hydroagg, workloads, dev, stream):
    """3000 sub-grids of mixed edges (polytrope), one hipGraph launch per step
    (eager launches timed beside it)."""
    dx = 0.5
    log("uneven: generating 3000 polytrope sub-grids")
    groups = workloads.polytrope(count=args.uneven_count, seed=3)
    tensors, descs, interiors, cells, tile_bytes = [], [], [], 0, 0
    for N, levels, U, _ in groups:
        t_in = torch.from_numpy(U).to(dev)
        t_out = t_in.clone()
        tensors.append((N, levels, t_in, t_out))
        # the step's output: updated interiors [F][n][n][n], as in the headline
        t_int = torch.empty((U.shape[0], U.shape[1], N, N, N), dtype=torch.float64, device=dev)
        interiors.append(t_int)
        descs.append(hydroagg.subgrids(t_in, t_int, levels=levels))
        cells += U.shape[0] * N ** 3
        tile_bytes += U.shape[0] * bytes_per_subgrid(N, U.shape[1])[1]
    batch = hydroagg.concat(*descs)
    count = batch[1]
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    plan = hydroagg.Plan(batch)
    plan.step(0.0, dx, amax, stream)
    torch.cuda.synchronize()
    lv = torch.cat([torch.as_tensor(l, dtype=torch.float64) for _, l, _, _ in tensors]).to(dev)
    dt = float(0.4 * torch.min(dx * torch.pow(2.0, -lv) / amax))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def back_to_back(fn, k):
        # untimed warm-up of at least --settle-ms, as for the headline: the
        # previous legs leave the GPU on other clocks
        t_warm = time.perf_counter()
        while True:
            for _ in range(3):
                fn()
            torch.cuda.synchronize()
            if (time.perf_counter() - t_warm) * 1e3 >= args.settle_ms:
                break
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    # the step (the amax-slot clear and one multi-class launch) replayed as
    # one hipGraph launch, and as eager launches beside it
    ms = back_to_back(lambda: plan.graph(dt, dx, amax, stream), args.uneven_steps)
    eager_ms = back_to_back(lambda: plan.step(dt, dx, amax, stream), args.uneven_steps)
    # each edge class alone: its own plan, eager launches (the class's kernel)
    per_class = {}
    if not args.no_uneven_classes:
        for (N, _, t_in, _), d in zip(tensors, descs):
            cplan = hydroagg.Plan(d)
            camax = torch.zeros(d[1], dtype=torch.float64, device=dev)
            cms = back_to_back(lambda: cplan.step(dt, dx, camax, stream), args.uneven_steps)
            cplan.close()
            ccells = int(t_in.shape[0]) * N ** 3
            per_class[int(N)] = {"subgrids": int(t_in.shape[0]), "us_per_step": round(cms * 1e3, 2),
                                 "value": round(ccells / (cms * 1e-3), 1)}
            log(f"uneven: class {N}^3 alone ({t_in.shape[0]} sub-grids): {cms * 1e3:.1f} us/step, "
                f"{ccells / cms / 1e6:.3f} G cell-updates/s")
    each_ms = None
    if args.uneven_each:
        e0.record(stream)
        hydroagg.hydro_step_each(batch, dt, dx, amax, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        each_ms = e0.elapsed_time(e1)
    plan.close()
    del interiors
    mix = {int(N): int(t.shape[0]) for N, _, t, _ in tensors}
    log(f"uneven: {ms * 1e3:.1f} us/step, {cells / ms / 1e6:.3f} G cell-updates/s; "
        f"per-sub-grid launches {each_ms} ms")
    res = {
        "workload": f"{count} polytrope sub-grids, edges {mix}, 11 FP64 fields, random octree "
                    "levels 2-5, one hipGraph launch per step (an amax-slot clear and one "
                    "multi-class kernel), updated interiors written [F][n][n][n]",
        "value": round(cells / (ms * 1e-3), 1), "unit": "cell-updates/s",
        "ms_per_step": round(ms, 5), "cells": cells,
        "eager_ms_per_step": round(eager_ms, 5),
        "achieved_gbs": round(tile_bytes / (ms * 1e-3) / 1e9, 1),
        "frac": round(tile_bytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "per_subgrid_launch": None if each_ms is None else {
            "ms_per_step": round(each_ms, 3), "value": round(cells / (each_ms * 1e-3), 1)},
        "aggregation_speedup": None if each_ms is None else round(each_ms / ms, 2),
        "per_class_alone": per_class or None,
    }
    return res, tensors, dt, dx, groups


def region_leg(args, torch, hydroagg, workloads, dev):
    """Generic aggregation regions (Section V-D): independent host tasks, one
    8^3 sub-grid each, from a pool of host threads.  Through a region, tasks
    that arrive together form a team: one upload, one step launch and one
    download per team.  The baseline has the same threads and tasks, one
    hydro_step launch per task on the thread's stream.  Wall time of the
    whole batch (hydro_region_drive)."""
    count, nf, dt, dx = args.region_tasks, 11, 2e-3, 1.0 / 64
    U = workloads.random_smooth(count, n=8, nfields=nf, seed=12)
    u_in = torch.from_numpy(U).to(dev)
    out = torch.empty((count, nf, 8, 8, 8), dtype=torch.float64, device=dev)
    descs = hydroagg.subgrids(u_in, out)
    rows = []
    for threads in args.region_threads:
        for mode, label in ((hydroagg.DRIVE_EACH, "one launch per task"),
                            (hydroagg.DRIVE_REGION, "region")):
            region = None
            if mode == hydroagg.DRIVE_REGION:
                region = hydroagg.Region(max_team=args.region_max_team, n_streams=2,
                                         arena_bytes=1 << 20)
            hydroagg.region_drive(region, (descs[0], min(count, 256)), dt, dx, threads, mode)
            secs = []
            for _ in range(args.region_reps):
                secs.append(hydroagg.region_drive(region, descs, dt, dx, threads, mode))
            row = {"mode": label, "threads": threads, "tasks": count,
                   "seconds": round(statistics.median(secs), 5),
                   "tasks_per_s": round(count / statistics.median(secs), 1)}
            if region is not None:
                st = region.stats()
                region.close()
                row["mean_team"] = round(st["tasks"] / max(st["teams"], 1), 2)
                row["launches"] = st["launches"]
            rows.append(row)
            log(f"regions: {label}, {threads} threads: {row['tasks_per_s'] / 1e3:.1f}k tasks/s"
                + (f", mean team {row['mean_team']}" if "mean_team" in row else ""))
    return {"workload": f"{count} independent tasks, each one 8^3 sub-grid with 11 FP64 fields "
                        "(random smooth), from a pool of host threads",
            "max_team": args.region_max_team, "rows": rows}


def timestep_leg(args, torch, hydroagg, workloads, dev, stream):
    """The paper's time-step shape (Table II: 512 sub-grids of 8^3 tiling a
    64^3 domain; three solver iterations per step, Section VI-A): one SSP-RK3
    time-step -- 3 aggregated stage kernels, each with its stage combination
    and face-ghost writes in its stores -- as ONE hipGraph launch on the
    device-resident brick."""
    per_axis, n, nf = 8, 8, args.nfields
    log(f"time-step: {per_axis ** 3} sub-grids of {n}^3, F={nf}, periodic brick")
    U = workloads.brick(seed=7, n=n, per_axis=per_axis, nfields=nf)
    count = U.shape[0]
    dx = 1.0 / (per_axis * n)
    u = torch.from_numpy(U).to(dev)
    w, s_ = torch.empty_like(u), torch.empty_like(u)
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    probe = torch.empty_like(u)
    hydroagg.hydro_step(hydroagg.subgrids(u, probe), 0.0, dx, amax, stream)
    torch.cuda.synchronize()
    dt = 0.4 * dx / float(amax.max())
    del probe
    rk = hydroagg.RK3(hydroagg.brick(n, nf, (per_axis,) * 3, (0, 0, 0)), u, w, s_)
    for _ in range(max(args.warmup, 5)):
        rk.graph(dt, dx, amax, stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.timestep_steps):
        rk.graph(dt, dx, amax, stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.timestep_steps
    rk.close()
    cells = count * n ** 3
    log(f"time-step: {ms * 1e3:.1f} us per SSP-RK3 step ({cells / (ms * 1e-3) / 1e6:.1f} M cell-steps/s)")
    return {"workload": f"{count} sub-grids of {n}^3 (+3 ghost layers) tiling a periodic "
                        f"{per_axis * n}^3 domain, {nf} FP64 fields, random smooth state",
            "what": "one SSP-RK3 time-step = 3 aggregated stage kernels (hydro step, stage "
                    "combination and face-ghost writes in one launch each), one hipGraph launch",
            "ms_per_timestep": round(ms, 5), "timesteps": args.timestep_steps,
            "cell_steps_per_s": round(cells / (ms * 1e-3), 1),
            "cell_updates_per_s": round(3 * cells / (ms * 1e-3), 1),
            "paper_context": "whole-application time per step of the 64^3 Sedov run: 86.6 ms "
                             "(A100, best aggregation), 130 ms (MI100); kernels, ghost exchange "
                             "and CPU work included there, device kernels only here"}


def strategies_leg(args, torch, hydroagg, workloads, dev, stream):
    """The paper's three aggregation strategies on this GPU (Section V, the
    parameter grid of Table III), on its scenario shape (Table II: 512
    sub-grids of 8^3, or 64 of 16^3 with the same cells), F = 11.  A
    time-step is three iterations; an iteration steps every sub-grid once.
    Strategy 1: 16^3 sub-grids, one launch each.  Strategy 2: 8^3 sub-grids,
    one launch each, dealt over k streams.  Strategy 3: the aggregator with
    max width W on one stream, every iteration's tasks arriving as a burst
    (aggregated while the stream is busy).  2+3: the aggregator with W and k
    streams.  Host wall time per time-step, median of --strategy-reps."""
    nf, dt, dx = args.nfields, 2e-3, 1.0 / 64
    u8 = torch.from_numpy(workloads.random_smooth(512, n=8, nfields=nf, seed=9)).to(dev)
    o8 = torch.empty((512, nf, 8, 8, 8), dtype=torch.float64, device=dev)
    u16 = torch.from_numpy(workloads.random_smooth(64, n=16, nfields=nf, seed=10)).to(dev)
    o16 = torch.empty((64, nf, 16, 16, 16), dtype=torch.float64, device=dev)
    d8 = hydroagg.subgrids(u8, o8)
    d16 = hydroagg.subgrids(u16, o16)
    cells = 512 * 8 ** 3

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.strategy_reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            ts.append((time.perf_counter() - t0) * 1e3)
        return round(statistics.median(ts), 3)

    def iters(step):
        def run():
            for _ in range(3):
                step()
        return run

    rows = []
    ms = timed(iters(lambda: hydroagg.hydro_step_each(d16, dt, dx, None, stream)))
    rows.append({"strategy": "1", "subgrid": "16^3", "executors": 1, "max_aggregated": 1,
                 "ms_per_timestep": ms})
    hydroagg.hydro_step_streams(d8, dt, dx, None, n_streams=max(args.strategy_streams), stream=stream)
    for k in args.strategy_streams:
        ms = timed(iters(lambda: hydroagg.hydro_step_streams(d8, dt, dx, None, n_streams=k,
                                                             stream=stream)))
        rows.append({"strategy": "2", "subgrid": "8^3", "executors": k, "max_aggregated": 1,
                     "ms_per_timestep": ms})

    def agg_row(label, width, k):
        agg = hydroagg.Aggregator(width, timeout_us=-1.0, n_streams=k, flush_when_idle=True)

        def it():
            agg.submit_many(d8, dt, dx)
            agg.drain()
        ms = timed(iters(it))
        st = agg.stats()
        agg.close()
        rows.append({"strategy": label, "subgrid": "8^3", "executors": k, "max_aggregated": width,
                     "ms_per_timestep": ms,
                     "mean_batch": round(st["launched"] / max(st["batches"], 1), 2)})

    for w in args.strategy_widths:
        agg_row("3", w, 1)
    for k, w in args.strategy_combos:
        agg_row("2+3", w, k)
    ms = timed(iters(lambda: hydroagg.hydro_step(d8, dt, dx, None, stream)))
    rows.append({"strategy": "one launch per iteration", "subgrid": "8^3", "executors": 1,
                 "max_aggregated": 512, "ms_per_timestep": ms})
    for r in rows:
        r["cell_updates_per_s"] = round(3 * cells / (r["ms_per_timestep"] * 1e-3), 1)
        log(f"strategy {r['strategy']}: {r['subgrid']}, {r['executors']} executors, max "
            f"aggregated {r['max_aggregated']}: {r['ms_per_timestep']} ms per time-step")
    base = next(r for r in rows if r["strategy"] == "2" and r["executors"] == 1)["ms_per_timestep"]
    s2 = [r for r in rows if r["strategy"] == "2"]
    s2_best = min(r["ms_per_timestep"] for r in s2)
    s2_max = max(s2, key=lambda r: r["executors"])["ms_per_timestep"]
    agg_rows = [r for r in rows if r["strategy"] in ("3", "2+3")]
    best = min(agg_rows, key=lambda r: r["ms_per_timestep"])
    return {"workload": "512 sub-grids of 8^3 (64 of 16^3 for strategy 1), 11 FP64 fields, "
                        "random smooth state, 3 iterations per time-step",
            "rows": rows,
            "best_aggregated": {k: best[k] for k in ("strategy", "executors", "max_aggregated",
                                                     "ms_per_timestep")},
            "speedup_best_vs_non_aggregated": round(base / best["ms_per_timestep"], 2),
            "speedup_best_vs_strategy2_most_streams": round(s2_max / best["ms_per_timestep"], 2),
            "speedup_best_vs_strategy2_best": round(s2_best / best["ms_per_timestep"], 2),
            "paper_context": "MI100 with HIP kernels (Table III): 1404 ms non-aggregated, 584 ms "
                             "with 128 executors, 166 ms strategy 3 (max 128), 130 ms best "
                             "combination (128 executors, max 16); 10.80x and 4.49x. Whole "
                             "application time per time-step there (5 kernels per sub-grid per "
                             "iteration, transfers, CPU work), the hydro kernel alone here"}


def step26_leg(args, torch, hydroagg, u_in, u_out, dt, dx, count, n, nf, stream):
    """The 26-point form (Section IV-B: 9 central-upwind flux points per face,
    Simpson's rule) on the headline batch and outputs; per-launch events."""
    descs = hydroagg.subgrids(u_in, u_out)
    for _ in range(2):
        hydroagg.hydro_step26(descs, dt, dx, None, stream)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.step26_reps)]
    for a_, b_ in ev:
        a_.record(stream)
        hydroagg.hydro_step26(descs, dt, dx, None, stream)
        b_.record(stream)
    torch.cuda.synchronize()
    ms = statistics.median(a_.elapsed_time(b_) for a_, b_ in ev)
    cells = count * n ** 3
    log(f"26-point step: {ms * 1e3:.1f} us per step ({cells / (ms * 1e-3) / 1e9:.3f} G cell-updates/s)")
    return {"workload": f"{count} sub-grids of {n}^3, {nf} FP64 fields, random smooth state, "
                        "updated interiors written [F][n][n][n]",
            "what": "26 reconstruction points per cell, 9 central-upwind flux points per face, "
                    "Simpson's rule over each face; one launch (descriptor copy included)",
            "ms_per_step": round(ms, 4), "value": round(cells / (ms * 1e-3), 1),
            "unit": "cell-updates/s", "flux_points_per_step": count * 3 * 9 * (n + 1) * n * n,
            "reps": args.step26_reps,
            "roofline": step26_roofline(hydroagg.version(), ms, count, n, nf)}


def step26_roofline(version, ms, count, n, nf):
    """The 26-point kernel is bound by vector ALU issue, not HBM (traffic
    1.4x its tile bytes in the committed profile): FP64 FLOP per launch and
    VALU instructions from the committed SQ counter record of this kernel
    build and workload (null otherwise), against the FP64 vector peak and
    against the issue time of those instructions on 256 CUs x 4 SIMDs at
    2.4 GHz (4 cycles per wave instruction)."""
    rec = counter_record("measured_fp64_step26.json", version,
                         f"{count}x{n}^3 F={nf} interior-out, 26-point form",
                         f"hydro_step26_kernel<{nf}>")
    if rec is None:
        return None
    tflops = float(rec["fp64_flop_per_launch"]) / (ms * 1e-3) / 1e12
    issue_ms = (float(rec["valu_insts_per_wave"]) * float(rec["waves_per_launch"]) * 4
                / (256 * 4 * 2.4e9) * 1e3)
    return {"bound": "alu", "achieved": round(tflops, 2), "peak": FP64_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(tflops / FP64_PEAK_TFLOPS, 4),
            "valu_issue_ms": round(issue_ms, 3), "valu_issue_frac": round(issue_ms / ms, 3)}


def _time_oracle(oracle, U, dt, dx, threads, seconds, levels=None, reps=2):
    """Median wall time of oracle.step over repetitions lasting >= seconds."""
    times = []
    t_all = time.time()
    while len(times) < reps or time.time() - t_all < seconds:
        t0 = time.time()
        oracle.step(U, dt, dx, levels=levels, nthreads=threads)
        times.append(time.time() - t0)
    return statistics.median(times), len(times), sum(times)


def cpu_baseline_leg(args, U, dt, dx, cells, poly):
    """The CPU oracle timed on the host cores: on all of them over the whole
    headline batch (the paper's 32-core row, Table III), on one thread over
    the first --cpu-single-count sub-grids (its 1-core row), and on all cores
    over the polytrope batch, with the limiter-branch and non-positive-state
    counters of one sequential pass over it."""
    import oracle
    threads = args.cpu_threads or int(os.environ.get("OMP_NUM_THREADS", "0") or 0) \
        or os.cpu_count() or 1
    count = U.shape[0]
    n = U.shape[2] - 2 * GHOST
    log(f"cpu baseline: oracle on the full batch, {threads} threads, >= {args.cpu_seconds:.0f} s")
    med, reps, wall = _time_oracle(oracle, U, dt, dx, threads, args.cpu_seconds)
    cpu = {"value": round(cells / med, 1), "unit": "cell-updates/s", "cores": threads,
           "kind": "oracle",
           "sample": f"the full {count}-sub-grid workload stepped {reps} times "
                     f"({wall:.1f} s wall, median {med:.3f} s per step), OpenMP over sub-grids"}
    log(f"cpu baseline {cells / med / 1e6:.2f} M cell-updates/s on {threads} threads")
    k = min(args.cpu_single_count, count)
    med1, reps1, wall1 = _time_oracle(oracle, U[:k], dt, dx, 1, args.cpu_single_seconds)
    c1 = k * n ** 3
    cpu["single_thread"] = {
        "value": round(c1 / med1, 1), "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
        "sample": f"the first {k} sub-grids of the workload stepped {reps1} times "
                  f"({wall1:.1f} s wall, median {med1:.3f} s per step), one thread"}
    log(f"cpu baseline {c1 / med1 / 1e6:.3f} M cell-updates/s on 1 thread")
    if poly is not None:
        groups, pdt, pdx = poly
        pcells = sum(G.shape[0] * N ** 3 for N, _, G, _ in groups)
        t_all, reps_p = 0.0, 0
        t_start = time.time()
        while reps_p < 2 or time.time() - t_start < args.cpu_uneven_seconds:
            t0 = time.time()
            for N, levels, G, _ in groups:
                oracle.step(G, pdt, pdx, levels=levels, nthreads=threads)
            t_all += time.time() - t0
            reps_p += 1
        counters = {}
        for N, levels, G, _ in groups:
            _, _, c = oracle.step(G, pdt, pdx, levels=levels, counters=True)
            for key, v in c.items():
                counters[key] = counters.get(key, 0) + int(v)
        cpu["uneven"] = {
            "value": round(pcells * reps_p / t_all, 1), "unit": "cell-updates/s", "cores": threads,
            "kind": "oracle",
            "sample": f"the {sum(G.shape[0] for _, _, G, _ in groups)}-sub-grid polytrope "
                      f"workload stepped {reps_p} times ({t_all:.1f} s wall)",
            "counters": counters,
            "counters_note": "one sequential oracle pass: cases of the limited slope and of the "
                             "parabola constraint taken, and cells / face states with rho <= 0 or "
                             "p <= 0 (the step has no floors)"}
        log(f"cpu baseline (polytrope) {pcells * reps_p / t_all / 1e6:.2f} M cell-updates/s; "
            f"counters {counters}")
    return cpu


def learned_leg(args, dev):
    """Width cost model trained on the GPU on the stored sweeps: held-out
    regret against the exhaustive tuner and the best static width."""
    from paper_2210_06438_amd import learned
    out = {"splits": args.learned_splits, "epochs": 2000, "features": 5,
           "overload_clip_us": learned.OVERLOAD_US,
           "exhaustive_runs_per_condition": len(learned.WIDTHS), "model_runs_per_condition": 0,
           "judge": "the model's width is run once; if that run falls behind the offered rate "
                    "(or the rate is outside the trained range) every width is run and the "
                    "best taken"}
    policies = {"timeout": "launch on width or 50 us timeout",
                "idle_r3": "launch on width, 50 us timeout or idle stream",
                "timeout_to2m": "launch on width or 50 us timeout; current runtime, rates to 2M/s"}
    for name in policies:
        recs = learned.load_sweep(name)
        t0 = time.time()
        cv = learned.cross_validate(recs, splits=range(args.learned_splits), device=dev)
        sec = time.time() - t0
        out[name] = {"policy": policies[name],
                     "model_mean_regret": round(cv["mlp_mean_regret"], 4),
                     "static_mean_regret": round(cv["static_mean_regret"], 4),
                     "model_median_regret": round(cv["mlp_median_regret"], 4),
                     "static_median_regret": round(cv["static_median_regret"], 4),
                     "static_widths": sorted({e["static_width"] for e in cv["splits"]}),
                     "model_wins": cv["mlp_wins"],
                     "judged_mean_regret": round(cv["judged_mean_regret"], 4),
                     "judged_median_regret": round(cv["judged_median_regret"], 4),
                     "judged_wins": cv["judged_wins"],
                     "judged_runs_per_condition": round(cv["judged_runs_per_condition"], 2),
                     "judged_fallbacks": cv["judged_fallbacks"], "conditions": cv["conditions"],
                     "train_seconds_per_model": round(sec / args.learned_splits, 3)}
        log(f"learned width ({name}): model regret mean {cv['mlp_mean_regret']:.3f} / median "
            f"{cv['mlp_median_regret']:.3f}; judged {cv['judged_mean_regret']:.3f} / "
            f"{cv['judged_median_regret']:.3f} at {cv['judged_runs_per_condition']:.2f} runs per "
            f"condition; best static {cv['static_mean_regret']:.3f} / "
            f"{cv['static_median_regret']:.3f}; wins model {cv['mlp_wins']}, judged "
            f"{cv['judged_wins']} of {args.learned_splits}; {sec / args.learned_splits:.2f} s per model")
    # the serving policy's width comes from the sweep that covers its rates
    model = learned.WidthModel(device=dev).fit(learned.load_sweep("timeout_to2m"))
    out["serving_model_sweep"] = "timeout_to2m"
    return out, model


def serving_leg(args, torch, hydroagg, np, tensors, dt, dx, dev, model=None):
    """Poisson arrivals of single-sub-grid tasks on the resident uneven pool;
    admission bounded by a fixed HBM budget of output slabs."""
    descs = [hydroagg.subgrids(t_in, t_out, levels=levels) for _, levels, t_in, t_out in tensors]
    pool = hydroagg.concat(*descs)
    edges = np.concatenate([np.full(t.shape[0], N) for N, _, t, _ in tensors])
    cells_of = edges.astype(np.int64) ** 3
    nfields = int(tensors[0][2].shape[1])
    size = {N: nfields * (N + 6) ** 3 * 8 for N in (8, 12, 16)}
    share = {N: float(np.sum(edges == N)) * size[N] for N in (8, 12, 16)}
    tot = sum(share.values())
    budget = args.serve_budget_mb * 2 ** 20
    arenas = []
    for N in (8, 12, 16):
        k = max(int(budget * share[N] / tot // size[N]), 1 if share[N] else 0)
        arenas.append((torch.zeros(max(k, 1) * size[N] // 8, dtype=torch.float64, device=dev), k))
    used = sum(k * size[N] for (t, k), N in zip(arenas, (8, 12, 16)))
    # the same bytes cut into interior-only slabs: (n/(n+6))^3 of the size each
    isize = {N: nfields * N ** 3 * 8 for N in (8, 12, 16)}
    iarenas = [(t, int(k * size[N] // isize[N])) for (t, k), N in zip(arenas, (8, 12, 16))]
    out = {"pool": int(len(edges)), "hbm_budget_bytes": int(used),
           "slabs": {N: k for (t, k), N in zip(arenas, (8, 12, 16))},
           "interior_slabs": {N: k for (t, k), N in zip(iarenas, (8, 12, 16))},
           "width": args.serve_width, "timeout_us": 50.0, "streams": args.serve_streams,
           "runs": []}
    rng = np.random.Generator(np.random.PCG64(4))
    for rate in args.serve_rates:
        n = int(rate * args.serve_seconds)
        task = rng.integers(0, len(edges), n).astype(np.int32)
        arrival = np.cumsum(rng.exponential(1e6 / rate, n))
        modes = [("aggregated", args.serve_width, True)]
        if rate <= args.per_task_max_rate:
            modes.append(("per_task_launch", 1, True))
        if rate >= 200000.0:
            modes.append(("aggregated_interior_slabs", args.serve_width, True))
        judged = None
        if model is not None:
            from paper_2210_06438_amd import learned
            mix = {int(N): float(np.mean(edges == N)) for N in (8, 12, 16)}
            # the judge's runs: the first tenth of the arrivals, at most 20000 tasks
            nj = max(400, min(n // 10, 20000))

            def measure(w):
                lat_j, _, _, st_j = hydroagg.serve_run(
                    pool, task[:nj], arrival[:nj], nfields=nfields, dt=dt, dx=dx,
                    slab_arenas=arenas, max_width=w, timeout_us=50.0,
                    n_streams=args.serve_streams, flush_when_idle=False)
                return {"width": w, "rate": rate, "p99_us": float(np.percentile(lat_j, 99)),
                        "throughput": nj / (max(st_j["makespan_us"], 1.0) * 1e-6)}
            jw, jruns, jhow = learned.JudgedWidth(model).choose(0, nfields, rate, measure, mix=mix)
            judged = {"model_width": model.choose_mix(mix, nfields, rate), "width": jw,
                      "judge_runs": jruns, "how": jhow, "judge_run_tasks": nj}
            modes.append(("timeout_policy_learned_width", jw, False))
        for label, width, idle in modes:
            inner = label == "aggregated_interior_slabs"
            lat, am, _, st = hydroagg.serve_run(
                pool, task, arrival, nfields=nfields, dt=dt, dx=dx,
                slab_arenas=iarenas if inner else arenas,
                max_width=width, timeout_us=50.0, n_streams=args.serve_streams,
                flush_when_idle=idle,
                out_layout=hydroagg.OUT_INTERIOR if inner else hydroagg.OUT_STORED)
            span = st["makespan_us"] * 1e-6
            rec = {"mode": label, "rate_per_s": rate, "tasks": n, "width": width,
                   "flush_when_idle": idle,
                   "p50_us": round(float(np.percentile(lat, 50)), 1),
                   "p99_us": round(float(np.percentile(lat, 99)), 1),
                   "mean_us": round(float(lat.mean()), 1),
                   "throughput_tasks_s": round(n / span, 1),
                   "cell_updates_s": round(float(cells_of[task].sum()) / span, 1),
                   "batches": st["agg"]["batches"],
                   "mean_batch": round(n / max(st["agg"]["batches"], 1), 2),
                   "max_live": st["max_live"],
                   "host_us_per_batch": round(st["launch_host_us"] / max(st["agg"]["batches"], 1), 2),
                   "launch_share_of_makespan": round(st["launch_host_us"] / max(st["makespan_us"], 1e-9), 3)}
            if label == "timeout_policy_learned_width":
                rec["judge"] = judged
            out["runs"].append(rec)
            log(f"serving {label} at {rate}/s: p50 {rec['p50_us']} us, p99 {rec['p99_us']} us, "
                f"{rec['throughput_tasks_s']:.0f} tasks/s, mean batch {rec['mean_batch']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--settle-ms", type=float, default=300.0,
                    help="untimed warm-up continues (in rounds of --warmup steps) until this "
                         "much time has passed")
    ap.add_argument("--count", type=int, default=4096)
    ap.add_argument("--n", type=int, default=8)
    ap.add_argument("--nfields", type=int, default=11)
    ap.add_argument("--each-reps", type=int, default=3,
                    help="timed repetitions of the one-launch-per-sub-grid baseline")
    ap.add_argument("--cpu-reps", type=int, default=2)
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="minimum wall time of the all-cores oracle measurement")
    ap.add_argument("--cpu-single-count", type=int, default=256,
                    help="sub-grids of the workload the one-thread oracle measurement steps")
    ap.add_argument("--cpu-single-seconds", type=float, default=5.0,
                    help="minimum wall time of the one-thread oracle measurement")
    ap.add_argument("--cpu-uneven-seconds", type=float, default=3.0,
                    help="minimum wall time of the oracle on the polytrope workload")
    ap.add_argument("--copy-reps", type=int, default=10,
                    help="timed repetitions of a plain device copy of the input buffer")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--launch-samples", type=int, default=60,
                    help="headline launches timed one by one for the per-launch median")
    ap.add_argument("--no-uneven", action="store_true", help="skip the uneven-size leg")
    ap.add_argument("--no-uneven-classes", action="store_true",
                    help="skip timing each edge class of the uneven leg alone")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--uneven-count", type=int, default=3000)
    ap.add_argument("--uneven-steps", type=int, default=100)
    ap.add_argument("--uneven-each", type=int, default=1,
                    help="1: also time the uneven batch with one launch per sub-grid")
    ap.add_argument("--serve-rates", type=float, nargs="*", default=[20000.0, 200000.0, 2000000.0, 5000000.0])
    ap.add_argument("--per-task-max-rate", type=float, default=200000.0,
                    help="skip the per-task-launch baseline above this rate (it saturates "
                         "near 60k tasks/s)")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--serve-width", type=int, default=64)
    ap.add_argument("--serve-streams", type=int, default=2)
    ap.add_argument("--serve-budget-mb", type=float, default=64.0)
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-width leg")
    ap.add_argument("--tile-tune", type=int, default=1,
                    help="1: choose every class's tile with the autotuner first (else the defaults)")
    ap.add_argument("--tile-count", type=int, default=512,
                    help="sub-grids per class in the tile sweep")
    ap.add_argument("--stored-leg", type=int, default=1,
                    help="1: also time the headline step writing the stored (n+6)^3 layout")
    ap.add_argument("--pattern-leg", type=int, default=1,
                    help="1: also time the step's access pattern without its arithmetic")
    ap.add_argument("--learned-splits", type=int, default=10)
    ap.add_argument("--no-timestep", action="store_true", help="skip the SSP-RK3 time-step leg")
    ap.add_argument("--no-regions", action="store_true", help="skip the aggregation-region leg")
    ap.add_argument("--region-tasks", type=int, default=4096)
    ap.add_argument("--region-threads", type=lambda s: [int(x) for x in s.split(",")],
                    default=[4, 16, 64])
    ap.add_argument("--region-max-team", type=int, default=64)
    ap.add_argument("--region-reps", type=int, default=3)
    ap.add_argument("--no-strategies", action="store_true", help="skip the strategy comparison leg")
    ap.add_argument("--step26-reps", type=int, default=10,
                    help="timed launches of the 26-point step (0: skip)")
    ap.add_argument("--strategy-reps", type=int, default=3)
    ap.add_argument("--strategy-streams", type=int, nargs="*",
                    default=[1, 2, 4, 8, 16, 32, 64, 128])
    ap.add_argument("--strategy-widths", type=int, nargs="*",
                    default=[1, 2, 4, 8, 16, 32, 64, 128])
    ap.add_argument("--strategy-combos", type=lambda v: tuple(int(x) for x in v.split("x")),
                    nargs="*", default=[(64, 8), (128, 8), (128, 16), (128, 32), (4, 16), (8, 32)],
                    help="streams x width pairs of the 2+3 combination, e.g. 128x16")
    ap.add_argument("--timestep-steps", type=int, default=50)
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
    # the step's output: each sub-grid's updated interior, [F][n][n][n] (the
    # interior-only layout; the stored (n+6)^3 layout is timed beside it)
    u_out = torch.empty((count, nf, n, n, n), dtype=torch.float64, device=dev)
    amax = torch.zeros(count, dtype=torch.float64, device=dev)
    descs = hydroagg.subgrids(u_in, u_out)
    plan = hydroagg.Plan(descs)
    stream = torch.cuda.current_stream()

    # ---- tile of every shape class, from the autotuner ---------------------
    # (after the host-side input generation, so the GPU comes to the timed
    # region straight from the sweep's work instead of from seconds idle)
    from paper_2210_06438_amd import tune
    tiles = None
    if args.tile_tune:
        recs, best = tune.tile_sweep(count=args.tile_count, dev=dev, log=log)
        tiles = {"chosen": {f"{k[0]}^3 F={k[1]}": v for k, v in best.items()}, "records": recs,
                 "batch": args.tile_count}

    plan.step(0.0, dx, amax, stream)
    torch.cuda.synchronize()
    dt = 0.4 * dx / float(amax.max())
    log(f"dt = {dt:.6e}; library {hydroagg.version()}")

    # ---- aggregated: one launch of the plan's kernel per step --------------
    # untimed warm-up: --warmup steps, continued until --settle-ms have
    # passed, so that the timed steps do not start on clocks still rising
    # from the light load of the tile sweep (a few steps are not enough)
    settle_steps = 0
    t_warm = time.perf_counter()
    while True:
        for _ in range(max(args.warmup, 1)):
            plan.step(dt, dx, amax, stream)
            settle_steps += 1
        torch.cuda.synchronize()
        if (time.perf_counter() - t_warm) * 1e3 >= args.settle_ms:
            break
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    def back_to_back(fn, k):
        """Mean duration of k back-to-back calls on the stream: one HIP event
        pair around the whole run (no markers between the launches)."""
        e0.record(stream)
        for _ in range(k):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / k

    ms = back_to_back(lambda: plan.step(dt, dx, amax, stream), args.steps)
    cells = count * n ** 3
    value = cells / (ms * 1e-3)
    log(f"aggregated: {ms * 1e3:.1f} us/step, {value / 1e9:.3f} G cell-updates/s")
    # The plan's step is this one kernel, so the timed region's mean is the
    # kernel's average launch duration (plus the small dispatch gap between
    # back-to-back launches): the roofline's denominator.
    kernel_ms = ms

    # ---- per-launch durations: the same step, each launch between its own
    # event pair (reported beside the value, which stays the timed region's
    # mean)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.launch_samples)]
    for a_, b_ in evs:
        a_.record(stream)
        plan.step(dt, dx, amax, stream)
        b_.record(stream)
    torch.cuda.synchronize()
    lat = sorted(1e3 * a_.elapsed_time(b_) for a_, b_ in evs)
    launch_durations = None if not lat else {
        "launches": len(lat), "median_us": round(statistics.median(lat), 2),
        "min_us": round(lat[0], 2), "max_us": round(lat[-1], 2)}
    if lat:
        log(f"per-launch durations: median {launch_durations['median_us']} us over {len(lat)} "
            f"launches (min {launch_durations['min_us']}, max {launch_durations['max_us']})")

    # ---- the same batch replayed as one hipGraph launch per step -----------
    for _ in range(3):
        plan.graph(dt, dx, amax, stream)
    graph_ms = back_to_back(lambda: plan.graph(dt, dx, amax, stream), args.steps)
    log(f"graph replay: {graph_ms * 1e3:.1f} us/step")

    # ---- the step's data movement alone: the access pattern without the
    # arithmetic, at the step's occupancy and at the occupancy registers allow
    pattern = None
    if args.pattern_leg:
        pattern = {}
        for same, key in ((True, "same_occupancy_us"), (False, "register_limited_us")):
            for _ in range(3):
                plan.pattern_floor(same, stream)
            pattern[key] = round(1e3 * back_to_back(lambda: plan.pattern_floor(same, stream),
                                                    args.steps), 2)
        pattern["step_over_pattern"] = round(kernel_ms * 1e3 / pattern["same_occupancy_us"], 3)
        log(f"access pattern alone: {pattern['same_occupancy_us']} us at the step's occupancy, "
            f"{pattern['register_limited_us']} us with no LDS limit")

    # ---- the same step writing the stored (n+6)^3 layout (reported beside) --
    stored_ms = stored_kernel_ms = None
    if args.stored_leg:
        u_st = u_in.clone()
        plan_s = hydroagg.Plan(hydroagg.subgrids(u_in, u_st))
        for _ in range(args.warmup):
            plan_s.step(dt, dx, amax, stream)
        torch.cuda.synchronize()
        stored_ms = back_to_back(lambda: plan_s.step(dt, dx, amax, stream), args.steps)
        stored_kernel_ms = stored_ms
        plan_s.close()
        del u_st
        log(f"stored-layout outputs: {stored_ms * 1e3:.1f} us/step, kernel {stored_kernel_ms * 1e3:.1f} us")

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
        u_cp = torch.empty_like(u_in)
        u_cp.copy_(u_in)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.copy_reps):
            u_cp.copy_(u_in)
        e1.record(stream)
        torch.cuda.synchronize()
        del u_cp
        copy_ms = e0.elapsed_time(e1) / args.copy_reps
        copy_gbs = 2 * u_in.numel() * 8 / (copy_ms * 1e-3) / 1e9
        log(f"device copy of {u_in.numel() * 8 / 1e9:.2f} GB: {copy_ms * 1e3:.1f} us, {copy_gbs:.0f} GB/s")

    step26 = None
    if args.step26_reps > 0 and n == 8:
        step26 = step26_leg(args, torch, hydroagg, u_in, u_out, dt, dx, count, n, nf, stream)

    floor_b, tile_b = bytes_per_subgrid(n, nf)
    achieved = tile_b * count / (kernel_ms * 1e-3) / 1e9
    achieved_floor = floor_b * count / (kernel_ms * 1e-3) / 1e9
    version = hydroagg.version()
    workload_name = f"{count}x{n}^3 F={nf} interior-out"
    kname = (f"hydro_lds8_kernel<{nf},{n + 2 * GHOST}>" if hydroagg.get_tile(n, nf) == 8
             else f"hydro_q4_kernel<{nf},{n + 2 * GHOST}>")
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": measured_traffic(version, workload_name, kname),
        "kernel": kname,
        "kernel_version": version,
        "algorithmic_bytes_per_launch": tile_b * count,
        "bytes_definition": "stored (n+6)^3 tile read once + interior n^3 written once, 8 B x F per cell",
        "achieved_floor_gbs": round(achieved_floor, 1),
        "kernel_ms": round(kernel_ms, 5),
        "timing": "achieved = algorithmic bytes / mean launch duration of the kernel: one HIP "
                  "event pair on the launch stream around the --steps back-to-back launches "
                  "of the timed region (the step is this one kernel)",
        "floor_bytes_per_launch": floor_b * count,
        "measured_copy_gbs": None if copy_gbs is None else round(copy_gbs, 1),
        "fp64": measured_fp64(version, workload_name, kname, kernel_ms),
        "access_pattern_alone": pattern,
    }

    learned_res = model = None
    if not args.no_learned:
        learned_res, model = learned_leg(args, dev)

    uneven = serving = poly = None
    if not args.no_uneven or not args.no_serving:
        del u_in, u_out
        torch.cuda.empty_cache()
        uneven, tensors, udt, udx, groups = uneven_leg(args, torch, hydroagg, workloads, dev, stream)
        poly = (groups, udt, udx)
        if args.no_uneven:
            uneven = None
        if not args.no_serving:
            serving = serving_leg(args, torch, hydroagg, np, tensors, udt, udx, dev, model)

    timestep = None
    if not args.no_timestep:
        timestep = timestep_leg(args, torch, hydroagg, workloads, dev, stream)

    regions = None
    if not args.no_regions:
        regions = region_leg(args, torch, hydroagg, workloads, dev)

    strategies = None
    if not args.no_strategies:
        strategies = strategies_leg(args, torch, hydroagg, workloads, dev, stream)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline_leg(args, U, dt, dx, cells, poly)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "warmup_steps_run": settle_steps,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{count} sub-grids of {n}^3 (+3 ghost layers), {nf} FP64 fields, "
                        "random smooth state, one aggregated kernel launch per step, "
                        "updated interiors written [F][n][n][n]",
            "subgrids": count, "n": n, "nfields": nf, "dx": dx, "cfl": 0.4,
            "tile": hydroagg.get_tile(n, nf),
        },
        "per_subgrid_launch": None if each_ms is None else {
            "value": round(cells / (each_ms * 1e-3), 1), "ms_per_step": round(each_ms, 4),
            "launches_per_step": count},
        "aggregation_speedup": None if each_ms is None else round(each_ms / ms, 2),
        "launch_durations": launch_durations,
        "graph_replay": {"ms_per_step": round(graph_ms, 5),
                         "value": round(cells / (graph_ms * 1e-3), 1),
                         "note": "the same step captured once and replayed as one hipGraph "
                                 "launch per step"},
        "stored_output_layout": None if stored_ms is None else {
            "ms_per_step": round(stored_ms, 5), "value": round(cells / (stored_ms * 1e-3), 1),
            "kernel_ms": round(stored_kernel_ms, 5),
            "frac": round(tile_b * count / (stored_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "note": "same step and inputs, u_out in the stored (n+6)^3 layout of u_in with only "
                    "the interior written: each 64-byte interior row leaves the memory sectors "
                    "it shares with ghost cells partly written"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "uneven": uneven,
        "serving": serving,
        "learned_width": learned_res,
        "timestep": timestep,
        "regions": regions,
        "strategies": strategies,
        "step26": step26,
        "tile_autotune": tiles,
    }
    plan.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
