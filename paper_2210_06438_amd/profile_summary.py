"""Summarise rocprofv3 CSV output of bench.py runs into a short markdown
profile and the per-launch HBM traffic record the benchmark reports.

Inputs are the directories written by
  rocprofv3 --kernel-trace --stats --output-format csv -d KT -o run -- python3 bench.py ...
  rocprofv3 --pmc FETCH_SIZE --output-format csv -d FETCH -o run -- python3 bench.py ...
  rocprofv3 --pmc WRITE_SIZE --output-format csv -d WRITE -o run -- python3 bench.py ...
FETCH_SIZE and WRITE_SIZE (KiB per dispatch) are scaled by what the same
counters read for the plain device copy that bench.py runs on the input
buffer (known size), then reported per launch of the hydro kernel.
"""
from __future__ import annotations

import argparse
import csv
import json
import os
import statistics


def _rows(d, name):
    with open(os.path.join(d, name)) as f:
        return list(csv.DictReader(f))


def kernel_stats(kt_dir, match, grid=None):
    """Durations of the traced dispatches whose name contains `match` (and
    whose grid has `grid` work-items, when given)."""
    name, durs = None, []
    for r in _rows(kt_dir, "run_kernel_trace.csv"):
        if match in r["Kernel_Name"] and (grid is None or int(r["Grid_Size_X"]) == grid):
            name = r["Kernel_Name"]
            durs.append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    if not durs:
        raise SystemExit(f"kernel {match!r} (grid {grid}) not in kernel trace")
    return {"name": name, "calls": len(durs), "avg_ns": statistics.mean(durs),
            "min_ns": min(durs), "max_ns": max(durs), "median_ns": statistics.median(durs)}


def counter(d, match, name, grid=None):
    vals = [float(r["Counter_Value"]) for r in _rows(d, "run_counter_collection.csv")
            if match in r["Kernel_Name"] and r["Counter_Name"] == name
            and (grid is None or int(r["Grid_Size"]) == grid)]
    if not vals:
        raise SystemExit(f"no {name} for {match!r} (grid {grid}) in {d}")
    return vals


def calibration(fetch_dir, write_dir, copy_bytes):
    """Bytes per counted byte of FETCH_SIZE and WRITE_SIZE, from the plain
    device copy of known size in the same run."""
    f_c = max(counter(fetch_dir, "copyBuffer", "FETCH_SIZE"))
    w_c = max(counter(write_dir, "copyBuffer", "WRITE_SIZE"))
    return copy_bytes / (f_c * 1024.0), copy_bytes / (w_c * 1024.0)


def step_spans(kt_dir, parts, skip=0):
    """Wall span of every step of a multi-class launch whose class kernels
    run concurrently: the traced dispatches of the `parts` ((match, grid)
    pairs), in start order, cut into groups holding one dispatch of each
    part; span = last end - first start of a complete group.  The first
    `skip` complete groups are left out."""
    ev = []
    for r in _rows(kt_dir, "run_kernel_trace.csv"):
        for k, (match, grid) in enumerate(parts):
            if match in r["Kernel_Name"] and int(r["Grid_Size_X"]) == grid:
                ev.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), k))
    ev.sort()
    spans, group = [], {}
    for st, en, k in ev:
        if k in group:
            group = {}
        group[k] = (st, en)
        if len(group) == len(parts):
            spans.append(max(e for _, e in group.values()) - min(s_ for s_, _ in group.values()))
            group = {}
    spans = spans[skip:]
    if not spans:
        raise SystemExit("no complete step in the kernel trace")
    return spans


def main_step(argv):
    """Summary of one multi-class step: per class the counters and the
    kernel durations (which overlap), and the step's wall span."""
    ap = argparse.ArgumentParser(prog="profile_summary.py step")
    ap.add_argument("--kt", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--part", action="append", required=True,
                    help="MATCH|GRID|LAUNCH_BYTES|LABEL for one class kernel")
    ap.add_argument("--copy-bytes", type=float, required=True)
    ap.add_argument("--version", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True)
    ap.add_argument("--out", required=True)
    ap.add_argument("--skip", type=int, default=0,
                    help="leading steps left out of the span (e.g. an eager pass)")
    a = ap.parse_args(argv)
    f_scale, w_scale = calibration(a.fetch, a.write, a.copy_bytes)
    parts = [p.split("|") for p in a.part]
    rows, tot_alg, tot_traffic = [], 0.0, 0.0
    for match, grid, lb, label in parts:
        grid, lb = int(grid), float(lb)
        ks = kernel_stats(a.kt, match, grid)
        rd = statistics.median(counter(a.fetch, match, "FETCH_SIZE", grid)) * 1024.0 * f_scale
        wr = statistics.median(counter(a.write, match, "WRITE_SIZE", grid)) * 1024.0 * w_scale
        tot_alg += lb
        tot_traffic += rd + wr
        rows.append(f"| {label} | `{ks['name'].split('(')[0].replace('void ', '')}` | {grid} | "
                    f"{ks['avg_ns'] / 1e3:.1f} | {rd / 1e6:.1f} | {wr / 1e6:.1f} | "
                    f"{lb / 1e6:.1f} | {(rd + wr) / lb:.3f} |")
    spans = step_spans(a.kt, [(m, int(g)) for m, g, _, _ in parts], a.skip)
    avg = statistics.mean(spans) * 1e-9
    lines = [
        "# Multi-class step: class kernels as concurrent graph branches",
        "",
        f"- workload: {a.workload}",
        f"- library: `{a.version}`",
        f"- command: `{a.command}`",
        f"- counters: the same command with `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE`"
        " (one counter per run; counter runs serialise the dispatches)",
        f"- copy calibration (bytes per counted byte): read x{f_scale:.4f}, write x{w_scale:.4f}",
        "",
        "Per class (durations overlap: the classes run side by side):",
        "",
        "| class | kernel | grid | avg duration us | HBM read MB | HBM write MB | "
        "algorithmic MB | traffic / algorithmic |",
        "|---|---|---|---|---|---|---|---|",
        *rows,
        "",
        "Whole step (first start to last end of one dispatch of every class):",
        "",
        "| quantity | value |",
        "|---|---|",
        f"| steps | {len(spans)}" + (f" (the first {a.skip} left out)" if a.skip else "") + " |",
        f"| step span | {avg * 1e6:.1f} us (median {statistics.median(spans) / 1e3:.1f}, "
        f"min {min(spans) / 1e3:.1f}, max {max(spans) / 1e3:.1f}) |",
        f"| HBM traffic per step | {tot_traffic / 1e6:.1f} MB |",
        f"| algorithmic bytes per step | {tot_alg / 1e6:.1f} MB |",
        f"| traffic / algorithmic | {tot_traffic / tot_alg:.3f} |",
        f"| algorithmic GB/s at average span | {tot_alg / avg / 1e9:.0f} |",
        "",
    ]
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


CUS = 256   # compute units of an MI355X

PASS1 = ["SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_VALU_ADD_F64", "SQ_INSTS_VALU_MUL_F64",
         "SQ_INSTS_VALU_FMA_F64", "SQ_INSTS_VALU_TRANS_F64", "SQ_INSTS_LDS", "SQ_INSTS_SALU"]
PASS2 = ["SQ_WAVES", "SQ_BUSY_CYCLES", "SQ_WAVE_CYCLES", "SQ_ACTIVE_INST_VALU",
         "SQ_ACTIVE_INST_LDS", "SQ_WAIT_INST_LDS", "SQ_LDS_BANK_CONFLICT", "SQ_WAIT_INST_ANY"]


def main_sq(argv):
    """FP64 operation count and instruction mix of one kernel from two SQ
    counter runs, with the kernel's average duration from a kernel-trace run.
    SQ_INSTS_VALU_*_F64 count wave instructions; every lane of this kernel's
    arithmetic is active, so FLOP = 64 x (ADD + MUL + TRANS + 2 FMA).  FP64
    min/max/compare instructions are not floating-point operations and are
    not counted."""
    ap = argparse.ArgumentParser(prog="profile_summary.py sq")
    ap.add_argument("--kt", required=True)
    ap.add_argument("--sq1", required=True)
    ap.add_argument("--sq2", required=True)
    ap.add_argument("--kernel", required=True)
    ap.add_argument("--grid", type=int, required=True)
    ap.add_argument("--cells", type=float, required=True, help="cell updates per launch")
    ap.add_argument("--version", required=True)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True,
                    help="the profiled program (what follows -- in both counter passes)")
    ap.add_argument("--kt-command", required=True, help="the kernel-trace command")
    ap.add_argument("--out", required=True)
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)

    def c(d, name):
        return statistics.median(counter(d, a.kernel, name, a.grid))
    waves = c(a.sq1, "SQ_WAVES")
    add, mul, fma, trans = (c(a.sq1, f"SQ_INSTS_VALU_{k}_F64") for k in ("ADD", "MUL", "FMA", "TRANS"))
    valu, lds, salu = c(a.sq1, "SQ_INSTS_VALU"), c(a.sq1, "SQ_INSTS_LDS"), c(a.sq1, "SQ_INSTS_SALU")
    wave_q = c(a.sq2, "SQ_WAVE_CYCLES")
    valu_q = c(a.sq2, "SQ_ACTIVE_INST_VALU")
    lds_q, conf_q = c(a.sq2, "SQ_ACTIVE_INST_LDS"), c(a.sq2, "SQ_LDS_BANK_CONFLICT")
    ks = kernel_stats(a.kt, a.kernel, a.grid)
    flop = 64.0 * (add + mul + trans + 2.0 * fma)
    avg_s = ks["avg_ns"] * 1e-9
    tflops = flop / avg_s / 1e12
    lines = [
        f"# {ks['name']}: FP64 operations and instruction mix",
        "",
        f"- workload: {a.workload}",
        f"- library: `{a.version}`",
        f"- pass 1: `rocprofv3 --pmc {' '.join(PASS1)} --output-format csv -d gpurun_out/sq1 "
        f"-o run -- {a.command}`",
        f"- pass 2: `rocprofv3 --pmc {' '.join(PASS2)} --output-format csv -d gpurun_out/sq2 "
        f"-o run -- {a.command}`",
        f"- duration: `{a.kt_command}`",
        "- FLOP = 64 x (ADD + MUL + TRANS + 2 FMA) wave instructions (all lanes active); "
        "FP64 min/max/compare not counted",
        "",
        "| quantity | value |",
        "|---|---|",
        f"| waves per launch | {waves:.0f} |",
        f"| VALU instructions per wave | {valu / waves:.0f} |",
        f"| FP64 ADD / MUL / FMA / TRANS per wave | {add / waves:.0f} / {mul / waves:.0f} / "
        f"{fma / waves:.0f} / {trans / waves:.0f} |",
        f"| LDS / SALU instructions per wave | {lds / waves:.0f} / {salu / waves:.0f} |",
        f"| FP64 FLOP per launch | {flop / 1e9:.3f} G |",
        f"| FP64 FLOP per cell update | {flop / a.cells:.0f} |",
        f"| kernel average duration (trace) | {ks['avg_ns'] / 1e3:.1f} us |",
        f"| achieved FP64 rate | {tflops:.2f} TFLOP/s ({tflops / 78.6:.1%} of 78.6) |",
        f"| wave life (SQ_WAVE_CYCLES, read as 4-cycle units) | {wave_q / waves * 4 / 2.4e3:.1f} us at 2.4 GHz |",
        f"| VALU busy per wave (SQ_ACTIVE_INST_VALU) | {valu_q / waves * 4 / 2.4e3:.1f} us "
        f"({valu_q / wave_q:.0%} of its life) |",
        f"| LDS active per wave (SQ_ACTIVE_INST_LDS, 4-cycle units) | {lds_q / waves * 4:.0f} cycles |",
        f"| LDS bank-conflict stall (SQ_LDS_BANK_CONFLICT, counted per CU, summed over the "
        f"{CUS} CUs) | {conf_q:.3g} cycles per launch = {conf_q / CUS / 2.4e3:.1f} us per CU at "
        f"2.4 GHz ({conf_q / CUS / 2.4e3 / (ks['avg_ns'] / 1e3):.0%} of the launch) |",
        "",
    ]
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))
    if a.json:
        with open(a.json, "w") as f:
            json.dump({"kernel_version": a.version, "kernel": ks["name"], "workload": a.workload,
                       "fp64_flop_per_launch": flop, "valu_insts_per_wave": valu / waves,
                       "waves_per_launch": waves}, f, indent=1)
            f.write("\n")


def main():
    import sys
    if len(sys.argv) > 1 and sys.argv[1] == "step":
        return main_step(sys.argv[2:])
    if len(sys.argv) > 1 and sys.argv[1] == "sq":
        return main_sq(sys.argv[2:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--kt", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--kernel", required=True, help="substring of the hydro kernel name")
    ap.add_argument("--grid", type=int, default=None,
                    help="only dispatches with this many work-items")
    ap.add_argument("--copy-bytes", type=float, required=True,
                    help="bytes the plain copy reads (= bytes it writes)")
    ap.add_argument("--launch-bytes", type=float, required=True,
                    help="algorithmic bytes of one hydro launch")
    ap.add_argument("--version", required=True, help="hydro_version() of the profiled library")
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True, help="the profiled command line")
    ap.add_argument("--out", required=True)
    ap.add_argument("--traffic-json", default=None)
    a = ap.parse_args()

    ks = kernel_stats(a.kt, a.kernel, a.grid)
    f_h = statistics.median(counter(a.fetch, a.kernel, "FETCH_SIZE", a.grid))
    w_h = statistics.median(counter(a.write, a.kernel, "WRITE_SIZE", a.grid))
    f_scale, w_scale = calibration(a.fetch, a.write, a.copy_bytes)
    rd = f_h * 1024.0 * f_scale
    wr = w_h * 1024.0 * w_scale
    traffic = rd + wr
    avg_s = ks["avg_ns"] * 1e-9
    lines = [
        f"# {ks['name']}",
        "",
        f"- workload: {a.workload}",
        f"- library: `{a.version}`",
        f"- command: `{a.command}`",
        f"- counters: the same command with `--pmc FETCH_SIZE` and `--pmc WRITE_SIZE`"
        " (one counter per run)",
        "",
        "| quantity | value |",
        "|---|---|",
        f"| launches traced | {ks['calls']}" + (f" (grid {a.grid} work-items)" if a.grid else "") + " |",
        f"| average duration | {ks['avg_ns'] / 1e3:.1f} us (median {ks['median_ns'] / 1e3:.1f}, "
        f"min {ks['min_ns'] / 1e3:.1f}, max {ks['max_ns'] / 1e3:.1f}) |",
        f"| FETCH_SIZE per launch (raw) | {f_h:.0f} KiB |",
        f"| WRITE_SIZE per launch (raw) | {w_h:.0f} KiB |",
        f"| copy calibration (bytes per counted byte) | read x{f_scale:.4f}, write x{w_scale:.4f} |",
        f"| HBM read per launch | {rd / 1e6:.1f} MB |",
        f"| HBM write per launch | {wr / 1e6:.1f} MB |",
        f"| HBM traffic per launch | {traffic / 1e6:.1f} MB |",
        f"| algorithmic bytes per launch | {a.launch_bytes / 1e6:.1f} MB |",
        f"| traffic / algorithmic | {traffic / a.launch_bytes:.3f} |",
        f"| algorithmic GB/s at average duration | {a.launch_bytes / avg_s / 1e9:.0f} |",
        f"| traffic GB/s at average duration | {traffic / avg_s / 1e9:.0f} |",
        "",
    ]
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    with open(a.out, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))
    if a.traffic_json:
        with open(a.traffic_json, "w") as f:
            json.dump({"kernel_version": a.version, "kernel": ks["name"],
                       "workload": a.workload, "traffic_bytes_per_launch": traffic,
                       "read_bytes": rd, "write_bytes": wr,
                       "avg_duration_us": ks["avg_ns"] / 1e3}, f, indent=1)
            f.write("\n")


if __name__ == "__main__":
    main()
