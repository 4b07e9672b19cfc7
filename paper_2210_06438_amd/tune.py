"""Autotuners: the tile (block shape) of each shape class, and the
aggregation width -- exhaustive, and the timing sweep that feeds the learned
width model.

Tile: tile_sweep() times one aggregated step of a batch of every (n, F)
class with each tile (8^3 or 4^3 blocks; the same faces, results equal to
rounding) and keeps the faster one (hydro_set_tile).

A serving condition is (n, nfields, arrival rate).  For each condition the
tuner replays the same seeded Poisson arrival sequence through the serving
loop (hydro_serve_run) at every candidate width and keeps the width with the
lowest p99 task latency (ties -> smaller width).  This is the paper's
hand-tuned "max aggregated kernels" parameter (Section VI-B, Table III),
found by measurement instead.

    python -m paper_2210_06438_amd.tune --out width_sweep.json
runs the full sweep (widths 1..512 x edges 8/12/16 x 6/11 fields x rates
2k..200k/s) on the GPU.
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

WIDTHS = [1, 2, 4, 8, 16, 32, 64, 128, 256, 512]
EDGES = [8, 12, 16]
FIELDS = [6, 11]
RATES = [2000.0, 5000.0, 10000.0, 20000.0, 50000.0, 100000.0, 200000.0]


def task_bytes(n: int, nfields: int) -> int:
    """Algorithmic bytes of one task: stored tile read + interior written."""
    return ((n + 6) ** 3 + n ** 3) * nfields * 8


class Pool:
    """Resident sub-grids of one (n, nfields) class and output slab arenas."""

    def __init__(self, n, nfields, count=256, budget_mb=64.0, seed=50, dev="cuda:0"):
        import torch

        from . import hydroagg, workloads
        U = workloads.random_smooth(count, n=n, nfields=nfields, seed=seed + 100 * n + nfields)
        self.n, self.nfields = n, nfields
        self.u_in = torch.from_numpy(U).to(dev)
        self.u_out = self.u_in.clone()
        self.descs = hydroagg.subgrids(self.u_in, self.u_out)
        words = nfields * (n + 6) ** 3
        k = max(1, int(budget_mb * 2 ** 20 // (words * 8)))
        self.arena = torch.zeros(k * words, dtype=torch.float64, device=dev)
        self.slabs = k
        self.count = count

    def arenas(self):
        return [(self.arena if e == self.n else None, self.slabs if e == self.n else 0)
                for e in EDGES]


TILES = (8, 4)


def tile_sweep(count=512, reps=20, warmup=3, seed=60, edges=EDGES, fields=FIELDS,
               dev="cuda:0", apply=True, log=None, rounds=3):
    """Time one aggregated step (a captured graph of the whole batch) of
    `count` random smooth sub-grids per class with each tile; returns
    (records, {(n, F): best tile}) and sets the best tiles when `apply`.
    The tiles are timed in turn for `rounds` rounds and each keeps its median
    round, so a clock still rising at the start favours neither."""
    import torch

    from . import hydroagg, workloads
    recs, best = [], {}
    stream = torch.cuda.current_stream()
    for n in edges:
        for nf in fields:
            U = workloads.random_smooth(count, n=n, nfields=nf, seed=seed + 100 * n + nf)
            u_in = torch.from_numpy(U).to(dev)
            u_out = u_in.clone()
            amax = torch.zeros(count, dtype=torch.float64, device=dev)
            plan = hydroagg.Plan(hydroagg.subgrids(u_in, u_out))
            before = hydroagg.get_tile(n, nf)
            runs = {tile: [] for tile in TILES}
            for _ in range(rounds):
                for tile in TILES:
                    hydroagg.set_tile(n, nf, tile)
                    for _ in range(warmup):
                        plan.graph(1e-4, 1.0 / 64, amax, stream)
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    for _ in range(reps):
                        plan.graph(1e-4, 1.0 / 64, amax, stream)
                    e1.record(stream)
                    torch.cuda.synchronize()
                    runs[tile].append(e0.elapsed_time(e1) / reps * 1e3)
            times = {tile: sorted(r)[len(r) // 2] for tile, r in runs.items()}
            for tile in TILES:
                recs.append({"n": n, "nfields": nf, "tile": tile, "count": count,
                             "us_per_step": round(times[tile], 2),
                             "rounds_us": [round(x, 2) for x in runs[tile]]})
            plan.close()
            best[(n, nf)] = min(times, key=lambda k: (times[k], -k))
            hydroagg.set_tile(n, nf, best[(n, nf)] if apply else before)
            if log:
                log(f"tile n={n} F={nf}: " + ", ".join(f"{k}^3 {v:.1f} us" for k, v in times.items())
                    + f" -> {best[(n, nf)]}^3")
            del u_in, u_out, U
    return recs, best


def run_condition(pool, rate, widths, *, seconds=0.2, min_tasks=400, streams=2,
                  timeout_us=50.0, seed=0, dt=1e-4, dx=1.0 / 64, flush_when_idle=False,
                  repeats=1):
    """Serve `repeats` independent arrival sequences at each width; one
    record per width, with the median over the repeats (p99_us) and each
    repeat's p99 (p99_runs_us)."""
    import numpy as np

    from . import hydroagg
    ntask = max(min_tasks, int(rate * seconds))
    seqs = []
    for r in range(repeats):
        rng = np.random.Generator(np.random.PCG64([seed + 1000 * r, pool.n, pool.nfields, int(rate)]))
        task = rng.integers(0, pool.count, ntask).astype(np.int32)
        seqs.append((task, np.cumsum(rng.exponential(1e6 / rate, ntask))))
    out = []
    for w in widths:
        runs = []
        for task, arrival in seqs:
            lat, _, _, st = hydroagg.serve_run(pool.descs, task, arrival, nfields=pool.nfields,
                                               dt=dt, dx=dx, slab_arenas=pool.arenas(),
                                               max_width=w, timeout_us=timeout_us,
                                               n_streams=streams, flush_when_idle=flush_when_idle)
            span = max(st["makespan_us"], 1.0) * 1e-6
            runs.append((float(np.percentile(lat, 50)), float(np.percentile(lat, 99)),
                         float(lat.mean()), ntask / span, st["agg"]["batches"]))
        med = [float(np.median([r[k] for r in runs])) for k in range(5)]
        out.append({"n": pool.n, "nfields": pool.nfields, "rate": rate, "width": w,
                    "streams": streams, "tasks": ntask, "flush_when_idle": bool(flush_when_idle),
                    "p50_us": med[0], "p99_us": med[1], "mean_us": med[2], "throughput": med[3],
                    "batches": int(med[4]), "repeats": repeats,
                    "p99_runs_us": [round(r[1], 2) for r in runs]})
    return out


def best_width(records):
    """{(n, nfields, rate): (width, p99)} of the lowest p99 (ties: smaller width)."""
    best = {}
    for r in records:
        key = (r["n"], r["nfields"], r["rate"])
        cand = (r["p99_us"], r["width"])
        if key not in best or cand < best[key]:
            best[key] = cand
    return {k: (w, p) for k, (p, w) in best.items()}


def exhaustive(n, nfields, rate, widths=WIDTHS, **kw):
    """Tune one condition: the best width and the records that chose it."""
    pool = Pool(n, nfields)
    recs = run_condition(pool, rate, widths, **kw)
    (w, p), = best_width(recs).values()
    return w, recs


def sweep(edges=EDGES, fields=FIELDS, rates=RATES, widths=WIDTHS, log=None, **kw):
    records = []
    for n in edges:
        for nf in fields:
            pool = Pool(n, nf)
            for rate in rates:
                t0 = time.time()
                recs = run_condition(pool, rate, widths, **kw)
                records += recs
                if log:
                    b = best_width(recs)
                    log(f"n={n} F={nf} rate={rate:.0f}: best {list(b.values())[0]} "
                        f"({time.time() - t0:.1f} s)")
            del pool
    return records


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--seconds", type=float, default=0.4)
    ap.add_argument("--streams", type=int, default=2)
    ap.add_argument("--idle-flush", action="store_true",
                    help="also launch whenever a stream is idle (off: width and timeout only)")
    ap.add_argument("--repeats", type=int, default=1,
                    help="independent arrival sequences per point (median p99 recorded)")
    ap.add_argument("--rates", type=float, nargs="*", default=RATES,
                    help="offered task rates (tasks/s)")
    a = ap.parse_args(argv)
    t0 = time.time()
    recs = sweep(rates=a.rates, seconds=a.seconds, streams=a.streams, flush_when_idle=a.idle_flush,
                 repeats=a.repeats, log=lambda m: print(m, flush=True))
    with open(a.out, "w") as f:
        json.dump({"widths": WIDTHS, "edges": EDGES, "fields": FIELDS, "rates": list(a.rates),
                   "seconds": a.seconds, "streams": a.streams, "timeout_us": 50.0,
                   "flush_when_idle": a.idle_flush, "slab_budget_mb": 64.0,
                   "repeats": a.repeats,
                   "records": recs}, f)
    print(f"{len(recs)} records in {time.time() - t0:.0f} s -> {a.out}", flush=True)


if __name__ == "__main__":
    sys.exit(main())
