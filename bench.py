#!/usr/bin/env python3
"""Throughput of the sketched matrix-profile discord path on one MI355X.

One step = the whole hot path over one batch of synthetic input already
resident in HBM: sketch_build (per-dimension statistics + projection),
mp_selfjoin (window statistics, self-join tiles, merge + FP64 polish) and
top_discords (top 10).  The workload is the water-treatment-shaped series:
d = 51 (25 AR(1) sensors, 26 on/off actuators), n = 50,000, Gaussian sketch
k = 8, m = 100, exclusion zone 25, three planted discords.

Metric: matrix-profile cells per second, cells = k * n^2 / 2 per step.
Prints ONE JSON line (rank 0).  Extra keys: ``roofline`` for the self-join
tile kernel (its own device time from HIP events on the library's stream),
``cpu_baseline`` (the CPU oracle on a bounded row sample), ``paths`` (each
precision measured).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X: 256 CUs x 4 SIMD x 16 lanes at 2.4 GHz = 3.93e13 VALU lane-ops/s
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9
OPS_PER_CELL_FP64 = 6  # 2 FMA (recurrence) + 2 MUL (normalisation) + 2 MAX (row, column)


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--workload", default="c1", choices=["c0", "c1", "c2", "c4"])
    ap.add_argument("--refresh", type=int, default=0,
                    help="mixed paths: rows between exact FP64 recomputations (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def _valid_half_pairs(n_sub: int, excl: int) -> int:
    L = max(0, n_sub - excl)
    return L * (L + 1) // 2


def _cpu_baseline(R_np, w, target_s: float):
    """The plain-C FP64 brute-force oracle, timed on a bounded sample of rows."""
    import numpy as np
    from oracle import c_oracle
    c = c_oracle()
    k, n = R_np.shape
    n_sub = n - w.m + 1
    rng = np.random.default_rng(0)
    c.profile(R_np[0], w.m, w.excl, rows=rng.choice(n_sub, 8, replace=False))   # warm-up
    t0 = time.perf_counter()
    c.profile(R_np[0], w.m, w.excl, rows=rng.choice(n_sub, 64, replace=False))
    per_row = max(time.perf_counter() - t0, 1e-4) / 64
    rows_per_group = max(4, min(n_sub, int(target_s / per_row / k)))
    total_rows = 0
    t0 = time.perf_counter()
    for g in range(k):
        rows = rng.choice(n_sub, rows_per_group, replace=False)
        c.profile(R_np[g], w.m, w.excl, rows=rows)
        total_rows += rows_per_group
    t = time.perf_counter() - t0
    t_full = t * (k * n_sub) / total_rows
    cells = w.cells()
    return {
        "value": cells / t_full,
        "unit": "cells/s",
        "cores": c.threads(),
        "kind": "oracle",
        "sample": f"{total_rows} profile rows ({rows_per_group} per group x {k} groups) of {k * n_sub}, "
                  f"each a full O(n m) brute-force row; {t:.1f} s measured, full profile extrapolated "
                  f"to {t_full:.0f} s",
    }


def main() -> int:
    args = _parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the sketched self-join of one workload is measured on a single "
              "MI355X (multi-GPU sharding is described in DESIGN.md, not built)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import datagen
    import paper_2311_03393_amd as skmp

    dev = torch.device("cuda:0")
    w = datagen.make(args.workload)
    d, n = w.T.shape
    n_sub = n - w.m + 1
    T = torch.from_numpy(w.T).to(dev)
    k = w.k
    R = torch.empty((k, n), dtype=torch.float64, device=dev)
    stats = torch.empty((1, d, 2), dtype=torch.float64, device=dev)
    P = torch.empty((k, n), dtype=torch.float64, device=dev)
    I = torch.empty((k, n), dtype=torch.int64, device=dev)
    ws = torch.empty(skmp.mp_selfjoin_workspace(w.offsets, k, w.m, args.prec), dtype=torch.uint8, device=dev)
    out = (torch.empty((1, 10), dtype=torch.int64, device=dev), torch.empty((1, 10), dtype=torch.int32, device=dev),
           torch.empty((1, 10), dtype=torch.float64, device=dev), torch.empty((1,), dtype=torch.int32, device=dev))

    def step():
        skmp.sketch_build(T, w.offsets, k, w.kind, w.sketch_seed, dim_ids=w.dim_ids, R=R, stats=stats)
        skmp.mp_selfjoin(R, w.offsets, k, w.m, w.excl, prec=args.prec, refresh=args.refresh, P=P, I=I, workspace=ws)
        skmp.top_discords(P, w.offsets, k, w.m, 10, out=out)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    skmp.timing_enable(True)
    for st in skmp.TIMERS:
        skmp.timing_read(st, reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    skmp.timing_enable(False)
    stage = {st: skmp.timing_read(st, reset=True) for st in skmp.TIMERS}
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    cells = w.cells()
    value = cells / (ms_per_step * 1e-3)

    tiles_ms, tiles_n = stage["tiles"]
    tile_avg_s = tiles_ms / max(tiles_n, 1) * 1e-3
    valid = k * _valid_half_pairs(n_sub, w.excl)
    achieved = OPS_PER_CELL_FP64 * valid / tile_avg_s
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": VALU_LANE_OPS_PEAK / 1e12,
        "unit": "Tops/s",
        "frac": achieved / VALU_LANE_OPS_PEAK,
        "traffic": None,
        "kernel": "sj_fp64_kernel<8,256>" if args.prec == "fp64" else f"selfjoin tiles ({args.prec})",
        "per_launch": {"cells": valid, "ops_per_cell": OPS_PER_CELL_FP64, "avg_ms": tile_avg_s * 1e3,
                       "launches": tiles_n},
        "basis": "FP64 VALU issue: 256 CU x 64 lanes x 2.4 GHz lane-ops/s; 6 lane-ops per valid half-matrix cell",
    }
    top = [int(x) for x in out[0][0].cpu()]
    result = {
        "metric": "matrix-profile cells/sec (k*n^2/2 per s)",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.prec == "fp64" else args.prec,
        "data": "synthetic",
        "config": {"workload": f"water-treatment-shaped d={d} n={n} gaussian k={k} m={w.m} excl={w.excl}"
                               if args.workload == "c1" else f"{args.workload} d={d} n={n} k={k} m={w.m}",
                   "precision": args.prec, "refresh": args.refresh, "cells_per_step": cells, "valid_half_pairs": valid,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "stages_ms_per_step": {st: v[0] / max(args.steps, 1) for st, v in stage.items()},
        "top10": top,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = _cpu_baseline(R.cpu().numpy(), w, args.cpu_seconds)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
