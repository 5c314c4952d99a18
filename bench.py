#!/usr/bin/env python3
"""Throughput of the sketched matrix-profile discord path on one MI355X.

One step = the whole hot path over one batch of synthetic input already
resident in HBM: sketch_build (per-dimension statistics + projection),
mp_selfjoin (window statistics, self-join tiles, merge + FP64 polish) and
top_discords (top 10 per series).  Default workload: the water-treatment-shaped
series, d = 51 (25 AR(1) sensors, 26 on/off actuators), n = 50,000, Gaussian
sketch k = 8, m = 100, exclusion zone 25, three planted discords; its named
precision is the FP32 path with an exact FP64 refresh every 256 rows.  Other
workloads: random-walk-small (small FP64 case), transportation (d = 1024,
n = 131,072, m = 288), merchant-batch (4096 merchant-shaped series, d = 32, lengths
U[2048, 65536], FP32 input, k = 4, m = 64, generated on the GPU), large-series (d = 256,
n = 2^20, k = 32, m = 256).

Metric: matrix-profile cells per second, cells = k * n^2 / 2 per series per
step.  Prints ONE JSON line.  ``value`` is the named precision's throughput
over the K timed steps, each a replay of one step captured in a HIP graph
(every kernel of the step runs; ``--eager`` times eager calls instead); ``paths`` repeats the measurement for the FP64 path
(and any other precision asked for) on the same input, with each path's error
against the FP64 path.  ``roofline`` covers the named path's tile kernel,
timed with HIP events on the library's stream; ``cpu_baseline`` times the CPU
oracle on a bounded sample of rows; ``dim_detect`` times the dimension
detection (Algorithm 3) of the named path's top discord.

Other modes (not the headline): ``--join ab`` measures the AB-join of a
single-series workload's second half against its first half;
``--experiment random-walks`` runs the random-walk experiment of Section IV-A
(sketched vs exact discord: success rate and speedup per d).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Published MI355X peaks: FP32 vector 157.3 TFLOP/s, FP64 vector 78.6 TFLOP/s,
# dense BF16 / FP16 matrix 2.5 PFLOP/s.  The roofline of a diagonal tile
# kernel counts the method's 6 operations per valid half-matrix cell (2 FMA of
# the recurrence, 2 MUL of the normalisation, 2 MIN of the row and column
# reductions) as flops against the vector peak of the path's precision.
PUBLISHED_PEAK = {"fp64": 78.6e12, "fp32": 157.3e12}
OPS_PER_CELL = 6  # 2 FMA (recurrence) + 2 MUL (normalise) + 2 MIN/MAX (row, column)
# Issue-slot model (a separate, labelled reading, not the roofline): 256 CUs x
# 4 SIMDs at 2.4 GHz; FP64 arithmetic, integer and min/max instructions retire
# 16 lanes per clock per SIMD (3.93e13 lane-ops/s); FP32 FMA / MUL / ADD 32
# lanes per clock per SIMD without packed math (7.86e13).
VALU_LANE_OPS_PEAK = 256 * 64 * 2.4e9
VALU_FP32_FAST_PEAK = 2 * VALU_LANE_OPS_PEAK
# cells/s at which each path's per-cell mix saturates the VALU issue:
#   FP64: 6 single-rate ops -> 6 / 3.93e13 s per lane-cell;
#   FP32: 4 double-rate FP32 ops + 2 single-rate minima -> 4 / 7.86e13 + 2 / 3.93e13.
CELL_PEAK = {"fp64": VALU_LANE_OPS_PEAK / 6.0,
             "fp32": 1.0 / (4.0 / VALU_FP32_FAST_PEAK + 2.0 / VALU_LANE_OPS_PEAK)}
CELL_PEAK_BASIS = {
    "fp64": "issue model: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz = 3.93e13 FP64 lane-ops/s; a cell = 2 FMA + 2 MUL + "
            "2 MIN, all single rate -> 6.55e12 cells/s",
    "fp32": "issue model: FP32 FMA/MUL at 32 lanes/clk/SIMD (7.86e13/s), integer minima at 16 (3.93e13/s); a cell "
            "= 2 FMA + 2 MUL (FP32) + 2 MIN (u32) = 4 issue slots -> 9.83e12 cells/s",
}
MFMA_16BIT_PEAK = 2.5e15  # dense BF16 / FP16 matrix-core peak of MI355X, FLOP/s
NAMED = {"random-walk-small": ("fp64", 0), "water-treatment": ("fp32", 256), "transportation": ("bf16x3", 0), "merchant-batch": ("fp32", 256), "large-series": ("fp16x3", 0)}
DESCR = {
    "random-walk-small": "random-walk+sine d=8 n=4096 sum sketch k=1 m=64 excl=16",
    "water-treatment": "water-treatment-shaped d=51 n=50000 gaussian k=8 m=100 excl=25",
    "transportation": "transportation-shaped d=1024 n=131072 gaussian k=16 m=288 excl=72",
    "merchant-batch": "merchant-shaped batch 4096 series d=32 L~U[2048,65536] fp32 input gaussian k=4 m=64 excl=16",
    "large-series": "random-walk+sine d=256 n=1048576 gaussian k=32 m=256 excl=64",
}
KERNELS = {"fp64": "sj_fp64_kernel<8,256,2,2,false>", "fp32": "sj_fp32_kernel<16,256,2,4>",
           "bf16x3": "sj_blk_kernel<BF16X3,2>", "fp16x3": "sj_blk_kernel<FP16X3,2>"}
KERNELS_HANKEL = {"bf16x3": "sj_mfma_kernel<BF16X3>", "fp16x3": "sj_mfma_kernel<FP16X3>"}


def _mixed_form(refresh: int) -> str:
    """Form the library runs for BF16x3 / FP16x3: the blocked recurrence unless
    the refresh period is below its shortest (128 rows) or the Hankel variant is
    forced by SKMP_MIXED_VARIANT=0."""
    if os.environ.get("SKMP_MIXED_VARIANT") == "0" or 0 < refresh < 128:
        return "hankel"
    return "blocked"


def _mfma_flops_per_cell(form: str, m: int) -> float:
    """MFMA flops the 16-bit split forms execute per valid cell: three products
    (hi*hi, hi*lo, lo*hi) of depth 32 per 16 x 16 tile step (blocked: 3 x 2 x 32
    = 192 whatever m) or of depth m (Hankel-direct: 6 m)."""
    return 192.0 if form == "blocked" else 6.0 * m


def _parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="water-treatment", choices=["random-walk-small", "water-treatment", "transportation", "merchant-batch", "large-series"])
    ap.add_argument("--prec", default=None, choices=["fp64", "fp32", "bf16x3", "fp16x3"],
                    help="headline precision (default: the one the workload names)")
    ap.add_argument("--refresh", type=int, default=None,
                    help="mixed paths: rows between exact FP64 recomputations (default: the workload's)")
    ap.add_argument("--also", default=None,
                    help="comma-separated extra precisions measured into 'paths' (default: fp64 plus, where a "
                         "step takes well under a second, the other mixed forms)")
    ap.add_argument("--eager", action="store_true",
                    help="time eager steps (the default times replays of one step captured in a HIP graph; "
                         "stage timings always come from eager steps)")
    ap.add_argument("--graph", action="store_true", help="the default (kept for old command lines)")
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MB",
                    help="run one plain device copy of MB MiB before the steps (reference for HBM byte counters)")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the FP64 / FP32 launch configuration first (on up to 64 series of a batch)")
    ap.add_argument("--join", default="self", choices=["self", "ab"],
                    help="ab: AB-join of the second half of a single-series workload (test) against its first "
                         "half (train), as in the train/test procedure")
    ap.add_argument("--no-dims", action="store_true", help="skip the dimension-detection measurement")
    ap.add_argument("--stream", action="store_true",
                    help="measure the streaming path: appends of new samples (sketch + self-join update)")
    ap.add_argument("--batch-list", default="1,16,256,2048",
                    help="--stream: samples per append (the first of these is the line's value)")
    ap.add_argument("--experiment", default=None, choices=["random-walks"],
                    help="random-walks: the sketched vs exact discord experiment of Section IV-A")
    ap.add_argument("--trials", type=int, default=100)
    ap.add_argument("--dims-list", default="250,500,1000,2500,5000,7500,10000")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the oracle on every group of the workload (water-treatment: about 50 s on 16 cores)")
    return ap.parse_args()


def _traffic(kernel: str, workload: str):
    """HBM bytes per launch of the tile kernel from the committed rocprofv3
    counter summary (FETCH_SIZE + WRITE_SIZE, calibrated on a plain copy), or
    None when there is none for this kernel and workload or the kernel's source
    has changed since the counters were taken."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for p in ("selfjoin.hip", "selfjoin_blocked.hip", "skmp_common.hpp"):
        with open(os.path.join(ROOT, "paper_2311_03393_amd", "csrc", p), "rb") as f:
            h.update(f.read())
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        with open(path) as f:
            for line in f:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(x.split("=", 1) for x in line.split()[1:])
                if kv.get("kernel") == kernel and kv.get("workload") == workload:
                    if kv.get("source_sha256") != h.hexdigest():
                        return None
                    return {"fetch_bytes": float(kv["fetch_bytes"]), "write_bytes": float(kv["write_bytes"]),
                            "source": os.path.relpath(path, ROOT)}
    return None


def _valid_half_pairs(n_sub: int, excl: int) -> int:
    L = max(0, n_sub - excl)
    return L * (L + 1) // 2


def _roofline_vector(prec: str, cells: float, avg_ms: float, launches: int, kernel: str, tr) -> dict:
    """Roofline of a diagonal tile kernel: the method's 6 operations per valid
    cell, counted as flops, per second of the kernel's own average launch time,
    against the published vector peak of its precision.  The issue-slot model
    (how far the kernel is from what the VALU can issue for its instruction
    mix) is reported beside it, labelled as such."""
    t = avg_ms * 1e-3
    achieved = OPS_PER_CELL * cells / t
    peak = PUBLISHED_PEAK[prec]
    return {
        "bound": "alu", "achieved": achieved / 1e12, "peak": peak / 1e12, "unit": "TFLOP/s",
        "frac": achieved / peak,
        "traffic": (tr["fetch_bytes"] + tr["write_bytes"]) if tr else None, "traffic_detail": tr,
        "kernel": kernel,
        "per_launch": {"cells": cells, "flops_per_cell": OPS_PER_CELL, "avg_ms": avg_ms, "launches": launches},
        "basis": f"6 flops per valid half-matrix cell (2 FMA + 2 MUL + 2 MIN) over the tile kernel's average launch "
                 f"time, against the published MI355X {prec.upper()} vector peak {peak / 1e12:.1f} TFLOP/s",
        "issue_model": {"cells_per_s_bound": CELL_PEAK[prec], "frac": cells / t / CELL_PEAK[prec],
                        "basis": CELL_PEAK_BASIS[prec]},
    }


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(R_host_series, w, target_s: float, full: bool = False):
    """The plain-C FP64 brute-force oracle on the host cores.

    R_host_series: list of (series index, k x L host array).  When one whole
    group's profile of a series fits the time budget (estimated from a short
    row sample), whole profiles are timed, group after group, until the budget
    is spent (``full``: every group of every listed series); otherwise rows
    are drawn in batches of 256 from random (series, group) pairs.  The time
    per row of a series is proportional to its number of windows, and the
    whole workload's time is extrapolated from the measured rate (no
    extrapolation when every group of every series was timed)."""
    import numpy as np
    from oracle import c_oracle
    c = c_oracle()
    rng = np.random.default_rng(0)
    lens = w.lengths()
    n_sub_all = np.maximum(lens - w.m + 1, 0).astype(np.float64)
    work_all = w.k * float(np.sum(n_sub_all * n_sub_all))      # window-rows x windows of the whole workload
    first = R_host_series[0][1]
    n_first = first.shape[1] - w.m + 1
    rows = rng.choice(n_first, min(256, n_first), replace=False)
    c.profile(first[0], w.m, w.excl, rows=rows[:8])  # warm-up
    t0 = time.perf_counter()
    c.profile(first[0], w.m, w.excl, rows=rows)
    est_group = (time.perf_counter() - t0) / (rows.size * n_first) * n_first * n_first
    rows_done, win_rows, t = 0, 0.0, 0.0
    if full or est_group <= 1.5 * target_s:
        groups_done = 0
        for s, Rs in R_host_series:
            n_sub = Rs.shape[1] - w.m + 1
            for g in range(w.k):
                if not full and t >= target_s:
                    break
                t0 = time.perf_counter()
                c.profile(Rs[g], w.m, w.excl)
                t += time.perf_counter() - t0
                rows_done += n_sub
                win_rows += float(n_sub) * n_sub
                groups_done += 1
        whole = full and len(R_host_series) == len(lens)
        sample = (f"whole brute-force profiles of {groups_done} (series, group) pairs "
                  f"({groups_done} of {w.k * len(lens)}), {rows_done} rows, {t:.1f} s measured" +
                  ("" if whole else ", the whole workload extrapolated by its window-rows"))
    else:
        while t < target_s:
            s, Rs = R_host_series[int(rng.integers(len(R_host_series)))]
            n_sub = Rs.shape[1] - w.m + 1
            rows = rng.choice(n_sub, min(256, n_sub), replace=False)
            t0 = time.perf_counter()
            c.profile(Rs[int(rng.integers(w.k))], w.m, w.excl, rows=rows)
            t += time.perf_counter() - t0
            rows_done += rows.size
            win_rows += rows.size * n_sub
        sample = (f"{rows_done} profile rows (batches of 256 random rows of a random group of "
                  f"{len(R_host_series)} series), each a full O(n m) brute-force row; {t:.1f} s measured")
    t_full = t / win_rows * work_all
    return {
        "value": w.cells() / t_full,
        "unit": "cells/s",
        "cores": c.threads(),
        "cpu_model": _cpu_model(),
        "kind": "oracle",
        "sample": sample + f"; whole workload {t_full:.0f} s",
    }


def _progress(msg: str) -> None:
    print("[bench] " + msg, file=sys.stderr, flush=True)


def _experiment_random_walks(args) -> int:
    """Section IV-A on the GPU: random walks of length 10,000 with d dimensions,
    m = 100, k = ceil(sqrt(d)) (71, 87 and 100 at d = 5,000, 7,500, 10,000),
    count sketch (the paper's), `trials` seeded repetitions per d (the paper's
    100 by default).  Per trial:
      sketched: sketch_build -> mp_selfjoin over the k groups -> top discord
                (Algorithm 2) -> dim_detect over the discord's group
                (Algorithm 3), self-join setting with the m/4 exclusion zone;
      exact:    every dimension's own self-join profile (exact_profiles: the
                d dimensions as one batch) and its top discord.
    Success, two readings of "ranked within the top 0.01 %":
      pairs:       the sketched discord's exact score (its dimension's profile
                   at its start) ranks within the top 0.01 % of all d x n'
                   exact (dimension, subsequence) scores;
      subsequence: the subsequence's exact multidimensional score (its largest
                   exact score over the d dimensions) ranks within the top
                   0.01 % of the n' subsequences (at n' = 9,901: it is the
                   largest);
    ties counted in its favour; each reported for (j*, i*) of Algorithms 2-3
    and after the refinement (the top discord of dimension j*'s own
    self-join).  Speedup:
    exact time / sketched time, both end to end on the GPU in the same
    precision; the ranking always uses FP64 exact scores.  Score densities (the
    figure of Section IV-A): a 40-bin density of every exact score over [0,
    2 sqrt(m)], pooled over the trials, and per trial the exact discord's score
    and the exact scores of the sketched and refined discords."""
    import math

    import numpy as np
    import torch

    import paper_2311_03393_amd as skmp
    dev = torch.device("cuda:0")
    n, m = 10000, 100
    excl = m // 4
    prec = args.prec or "fp64"
    refresh = args.refresh if args.refresh is not None else 0
    ds = [int(x) for x in args.dims_list.split(",")]
    rows = []
    for d in ds:
        k = skmp.sketch_default_k(d)  # ceil(sqrt(d))
        succ, succ_ref, t_sk, t_ref, t_ex, ranks, ranks_ref = 0, 0, [], [], [], [], []
        succ_sub, succ_sub_ref, ranks_sub, ranks_sub_ref = 0, 0, [], []
        # score densities (the figure of Section IV-A at d = 1000): every exact score, pooled over the
        # trials, and per trial the exact discord's score and the sketched / refined discords' exact scores
        smax = 2.0 * math.sqrt(m)
        nbins = 40
        hist = torch.zeros(nbins, dtype=torch.float64, device=dev)
        s_exact, s_sketch, s_ref = [], [], []
        for trial in range(args.trials):
            seed = 7919 * d + trial
            g = torch.Generator(device=dev)
            g.manual_seed(seed)
            T = torch.randn((d, n), generator=g, dtype=torch.float64, device=dev).cumsum_(dim=1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            R, stats = skmp.sketch_build(T, [0, n], k, "count", seed)
            P, _ = skmp.mp_selfjoin(R, [0, n], k, m, excl, prec=prec, refresh=refresh)
            idx, grp, _, _ = skmp.top_discords(P, [0, n], k, m, 1)
            i_star, g_star = int(idx[0, 0].item()), int(grp[0, 0].item())
            dims = skmp.group_dims("count", k, seed, g_star, np.arange(d))
            _, _, best = skmp.dim_detect(T, stats[0], dims, i_star, m, excl=excl)
            j_star = int(dims[int(best.item())])
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            i_ref, _ = skmp.refine_discord(T, j_star, m, excl, prec=prec, refresh=refresh)
            torch.cuda.synchronize()
            t1r = time.perf_counter()
            Pe, _ = skmp.exact_profiles(T, m, excl, prec=prec, refresh=refresh)
            offs = np.arange(d + 1, dtype=np.int64) * n
            eidx, _, escore, _ = skmp.top_discords(Pe.reshape(1, d * n), offs, 1, m, 1)
            _ = int(torch.argmax(escore[:, 0]).item())   # the exact multidimensional discord
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            t_sk.append(t1 - t0)
            t_ref.append(t1r - t1)
            t_ex.append(t2 - t1r)
            if prec != "fp64":
                Pe, _ = skmp.exact_profiles(T, m, excl, prec="fp64")
            n_sub = n - m + 1
            scores = Pe[:, :n_sub]
            total = d * n_sub
            rank = int((scores > scores[j_star, i_star]).sum().item()) + 1
            rank_ref = int((scores > scores[j_star, i_ref]).sum().item()) + 1
            # subsequence reading: the multidimensional score max_j P_j[i], ranked over the n' subsequences
            A = torch.where(torch.isfinite(scores), scores, torch.full_like(scores, -math.inf)).max(dim=0).values
            rank_sub = int((A > A[i_star]).sum().item()) + 1
            rank_sub_ref = int((A > A[i_ref]).sum().item()) + 1
            top_sub = max(1, int(1e-4 * n_sub))
            succ_sub += int(rank_sub <= top_sub)
            succ_sub_ref += int(rank_sub_ref <= top_sub)
            ranks_sub.append(rank_sub / n_sub)
            ranks_sub_ref.append(rank_sub_ref / n_sub)
            hist += torch.histc(scores, bins=nbins, min=0.0, max=smax)
            s_exact.append(float(scores.max().item()))
            s_sketch.append(float(scores[j_star, i_star].item()))
            s_ref.append(float(scores[j_star, i_ref].item()))
            ranks.append(rank / total)
            ranks_ref.append(rank_ref / total)
            succ += int(rank <= 1e-4 * total)
            succ_ref += int(rank_ref <= 1e-4 * total)
            del T, R, stats, P, Pe, scores
            if (trial + 1) % 25 == 0 and trial + 1 < args.trials:
                _progress(f"random walks d={d}: {trial + 1} trials")
        tsk, tref, tex = float(np.median(t_sk)), float(np.median(t_ref)), float(np.median(t_ex))
        rows.append({"d": d, "k": k, "trials": args.trials, "success_rate": succ / args.trials,
                     "success_rate_refined": succ_ref / args.trials,
                     "median_rank_fraction": float(np.median(ranks)),
                     "median_rank_fraction_refined": float(np.median(ranks_ref)),
                     "success_rate_subsequence": succ_sub / args.trials,
                     "success_rate_subsequence_refined": succ_sub_ref / args.trials,
                     "median_rank_fraction_subsequence": float(np.median(ranks_sub)),
                     "median_rank_fraction_subsequence_refined": float(np.median(ranks_sub_ref)),
                     "t_sketched_ms": 1e3 * tsk, "t_refine_ms": 1e3 * tref, "t_exact_ms": 1e3 * tex,
                     "speedup": tex / tsk, "speedup_with_refinement": tex / (tsk + tref),
                     "score_density": {
                         "bin_edges": [smax * b / nbins for b in range(nbins + 1)],
                         "all_scores": (hist / (hist.sum() * (smax / nbins))).cpu().tolist(),
                         "exact_discord_scores": s_exact, "sketched_discord_scores": s_sketch,
                         "refined_discord_scores": s_ref}})
        _progress(f"random walks d={d} k={k}: success {succ}/{args.trials}, refined {succ_ref}/{args.trials}; "
                  f"subsequence reading {succ_sub}/{args.trials}, refined {succ_sub_ref}/{args.trials}; "
                  f"speedup {rows[-1]['speedup']:.1f}x ({rows[-1]['speedup_with_refinement']:.1f}x refined); "
                  f"median scores: exact discord {np.median(s_exact):.3f}, sketched {np.median(s_sketch):.3f}, "
                  f"refined {np.median(s_ref):.3f}")
    print(json.dumps({"experiment": "Section IV-A random walks: sketched vs exact discord", "n": n, "m": m,
                      "excl": excl, "precision": prec, "sketch": "count", "rows": rows}), flush=True)
    return 0


def _bench_ab(args, prec: str, refresh: int) -> int:
    """AB-join throughput: the second half of a single-series workload (test)
    against its first half (train).  One step sketches both halves, joins the
    test half against the train half and takes the test half's top-10
    discords.  Cells = k * na' * nb' (every pair of the rectangle)."""
    import numpy as np
    import torch

    import datagen
    import paper_2311_03393_amd as skmp
    if args.workload == "merchant-batch":
        print("the AB-join measurement takes a single-series workload (random-walk-small, water-treatment, transportation, large-series)", file=sys.stderr)
        return 2
    if prec not in ("fp64", "fp32"):
        prec, refresh = "fp32", 0
    dev = torch.device("cuda:0")
    w = datagen.make(args.workload)
    k, m = w.k, w.m
    n = w.T.shape[1]
    half = n // 2
    T = torch.from_numpy(w.T).to(dev)
    Ta, Tb = T[:, half:].contiguous(), T[:, :half].contiguous()
    del T
    na, nb = n - half, half
    na_sub, nb_sub = na - m + 1, nb - m + 1
    cells = float(k) * na_sub * nb_sub
    Ra = torch.empty((k, na), dtype=torch.float64, device=dev)
    Rb = torch.empty((k, nb), dtype=torch.float64, device=dev)
    sa = torch.empty((1, w.T.shape[0], 2), dtype=torch.float64, device=dev)
    sb = torch.empty_like(sa)
    PA = torch.empty((k, na), dtype=torch.float64, device=dev)
    IA = torch.empty((k, na), dtype=torch.int64, device=dev)
    out = (torch.empty((1, 10), dtype=torch.int64, device=dev), torch.empty((1, 10), dtype=torch.int32, device=dev),
           torch.empty((1, 10), dtype=torch.float64, device=dev), torch.empty((1,), dtype=torch.int32, device=dev))
    results, profiles, picks = {}, {}, {}

    def measure(pr: str, rf: int, steps: int, warmup: int):
        ws = torch.empty(max(skmp.mp_abjoin_workspace(na, nb, k, m, pr), 256), dtype=torch.uint8, device=dev)

        def step():
            skmp.sketch_build(Ta, [0, na], k, w.kind, w.sketch_seed, dim_ids=w.dim_ids, R=Ra, stats=sa)
            skmp.sketch_build(Tb, [0, nb], k, w.kind, w.sketch_seed, dim_ids=w.dim_ids, R=Rb, stats=sb)
            skmp.mp_abjoin(Ra, Rb, k, m, prec=pr, refresh=rf, PA=PA, IA=IA, workspace=ws)
            skmp.top_discords(PA, [0, na], k, m, 10, out=out)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        _progress(f"ab {pr}: {warmup} warmup step(s) done")
        skmp.timing_enable(True)
        for st in skmp.TIMERS:
            skmp.timing_read(st, reset=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        skmp.timing_enable(False)
        stage = {st: skmp.timing_read(st, reset=True) for st in skmp.TIMERS}
        ms = (t1 - t0) * 1e3 / steps
        _progress(f"ab {pr}: {steps} timed step(s), {ms:.3f} ms each")
        tiles_ms, tiles_n = stage["tiles"]
        tile_s = tiles_ms / max(tiles_n, 1) * 1e-3
        profiles[pr] = PA[:, :na_sub].clone()
        picks[pr] = out[0].cpu().clone()
        return {"precision": pr, "refresh": rf, "ms_per_step": ms, "cells_per_s": cells / (ms * 1e-3),
                "tile_kernel_ms": tile_s * 1e3, "tile_launches": tiles_n,
                "tile_frac_of_vector_peak": OPS_PER_CELL * cells / tile_s / PUBLISHED_PEAK[pr],
                "tile_frac_of_issue_model": cells / tile_s / CELL_PEAK[pr],
                "stages_ms_per_step": {st: v[0] / max(steps, 1) for st, v in stage.items()},
                "top10": [int(x) for x in out[0][0].cpu()]}

    head = measure(prec, refresh, args.steps, args.warmup)
    results[prec + (f"_refresh{refresh}" if refresh else "")] = head
    if prec != "fp64":
        results["fp64"] = measure("fp64", 0, max(3, args.steps // 2), 1)
        ref, got = profiles["fp64"], profiles[prec]
        head["vs_fp64"] = {"max_abs_dP": float((got - ref).abs().max()), "tolerance_dP": 1e-3 * 2 * m ** 0.5,
                           "top10_equal": bool(torch.equal(picks[prec], picks["fp64"]))}
    result = {
        "metric": "AB-join matrix-profile cells/sec (k*na'*nb' per s)",
        "value": head["cells_per_s"], "unit": "cells/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32"}[prec], "data": "synthetic",
        "config": {"workload": DESCR[args.workload] + ": test = second half, train = first half",
                   "precision": prec, "refresh": refresh, "na": na, "nb": nb, "cells_per_step": cells,
                   "parallelism": "single GPU"},
        "roofline": _roofline_vector(prec, cells, head["tile_kernel_ms"], head["tile_launches"], KERNELS[prec], None),
        "paths": results,
    }
    print(json.dumps(result), flush=True)
    return 0


def _bench_stream(args, prec: str, refresh: int) -> int:
    """Streaming (Section III-B's streaming extension): the first 80 % of a
    single-series workload is sketched and joined once; the rest arrives in
    appends of `a` samples, each sketched with the frozen statistics and
    merged into the profile by mp_selfjoin_append.  Per batch size: the
    latency of one append (synchronised), the pipelined time per append, the
    stage split, and the cost of recomputing the whole series instead."""
    import numpy as np
    import torch

    import datagen
    import paper_2311_03393_amd as skmp
    if args.workload == "merchant-batch":
        print("the streaming measurement takes a single-series workload (random-walk-small, water-treatment, transportation, large-series)", file=sys.stderr)
        return 2
    if prec not in ("fp64", "fp32"):
        prec, refresh = "fp32", 0
    dev = torch.device("cuda:0")
    w = datagen.make(args.workload)
    k, m, excl = w.k, w.m, w.excl
    d, n = w.T.shape
    n0 = (n * 4) // 5
    T = torch.from_numpy(w.T).to(dev)
    R = torch.empty((k, n), dtype=torch.float64, device=dev)
    P = torch.full((k, n), float("nan"), dtype=torch.float64, device=dev)
    I = torch.full((k, n), -2, dtype=torch.int64, device=dev)
    _, stats = skmp.sketch_build(T[:, :n0], [0, n0], k, w.kind, w.sketch_seed, dim_ids=w.dim_ids, R=R[:, :n0])
    skmp.mp_selfjoin(R[:, :n0], [0, n0], k, m, excl, prec=prec, refresh=refresh, P=P, I=I)
    torch.cuda.synchronize()
    P0, I0 = P.clone(), I.clone()
    ws_j = torch.empty(max(skmp.mp_selfjoin_append_workspace([n], k, m, prec), 256), dtype=torch.uint8, device=dev)

    # the alternative: sketch and join the whole series again
    Rf = torch.empty((k, n), dtype=torch.float64, device=dev)
    sf = torch.empty((1, d, 2), dtype=torch.float64, device=dev)
    Pf = torch.empty((k, n), dtype=torch.float64, device=dev)
    If = torch.empty((k, n), dtype=torch.int64, device=dev)
    ws_f = torch.empty(max(skmp.mp_selfjoin_workspace([0, n], k, m, prec), 256), dtype=torch.uint8, device=dev)

    def full():
        skmp.sketch_build(T, [0, n], k, w.kind, w.sketch_seed, dim_ids=w.dim_ids, R=Rf, stats=sf)
        skmp.mp_selfjoin(Rf, [0, n], k, m, excl, prec=prec, refresh=refresh, P=Pf, I=If, workspace=ws_f)

    full()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        full()
    torch.cuda.synchronize()
    full_ms = (time.perf_counter() - t0) * 1e3 / 3
    _progress(f"stream {prec}: full recompute {full_ms:.3f} ms")

    def append(cur: int, a: int):
        skmp.sketch_append(T[:, cur:cur + a], [0, a], [cur], R, stats, k, w.kind, w.sketch_seed, dim_ids=w.dim_ids)
        skmp.mp_selfjoin_append(R, P, I, [0], [cur], [cur + a], k, m, excl, prec=prec, refresh=refresh,
                                workspace=ws_j)

    def restore():
        P.copy_(P0)
        I.copy_(I0)

    batches = {}
    for a in [int(x) for x in args.batch_list.split(",") if x]:
        reps = max(1, min(max(args.steps, 100), (n - n0) // a))
        restore()
        append(n0, a)  # warm-up (plans, workspace)
        torch.cuda.synchronize()
        restore()
        torch.cuda.synchronize()
        lat = []
        cur = n0
        for _ in range(reps):
            t0 = time.perf_counter()
            append(cur, a)
            torch.cuda.synchronize()
            lat.append((time.perf_counter() - t0) * 1e3)
            cur += a
        # the stage split, from a pass with the stage timers on
        restore()
        skmp.timing_enable(True)
        for st in skmp.TIMERS:
            skmp.timing_read(st, reset=True)
        cur = n0
        for _ in range(reps):
            append(cur, a)
            cur += a
        torch.cuda.synchronize()
        skmp.timing_enable(False)
        stage = {st: skmp.timing_read(st, reset=True) for st in skmp.TIMERS}
        # pipelined appends (no timers)
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cur = n0
        for _ in range(reps):
            append(cur, a)
            cur += a
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / reps
        # the grown profile against a batch join of the same samples (same precision)
        Pb, Ib = skmp.mp_selfjoin(R[:, :cur], [0, cur], k, m, excl, prec=prec, refresh=refresh)
        torch.cuda.synchronize()
        n_sub = cur - m + 1
        dP = float((P[:, :n_sub] - Pb[:, :n_sub]).abs().max())
        same_I = float((I[:, :n_sub] == Ib[:, :n_sub]).double().mean())
        # pairs whose later subsequence is new: sum over new windows j of (j - excl + 1)
        j0, j1 = n0 - m + 1, cur - m + 1
        new_pairs = k * ((j1 - excl) * (j1 - excl + 1) - (j0 - excl) * (j0 - excl + 1)) / 2.0
        tiles_ms, tiles_n = stage["tiles"]
        _progress(f"stream {prec}: a={a}: {ms:.3f} ms per append (latency median {np.median(lat):.3f} ms)")
        batches[str(a)] = {
            "samples_per_append": a, "appends": reps, "ms_per_append": ms,
            "latency_ms": {"median": float(np.median(lat)), "max": float(np.max(lat))},
            "samples_per_s": a * reps / (ms * reps * 1e-3),
            "new_pairs_per_append": new_pairs / reps, "new_pairs_per_s": new_pairs / (ms * reps * 1e-3),
            "stages_ms_per_append": {st: v[0] / reps for st, v in stage.items() if v[1]},
            "tile_kernel_ms": tiles_ms / max(tiles_n, 1),
            "full_recompute_ms": full_ms, "speedup_vs_recompute": full_ms / ms,
            "vs_batch_join": {"max_abs_dP": dP, "same_neighbour_frac": same_I},
        }
    restore()
    first = batches[next(iter(batches))]
    result = {
        "metric": "streaming: appended samples per second (sketch + self-join update)",
        "value": first["samples_per_s"], "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": first["ms_per_append"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32"}[prec], "data": "synthetic",
        "config": {"workload": DESCR[args.workload] + f": first {n0} samples joined once, the rest appended",
                   "precision": prec, "refresh": refresh, "samples_per_append": first["samples_per_append"],
                   "parallelism": "single GPU"},
        "batches": batches,
    }
    print(json.dumps(result), flush=True)
    return 0


def main() -> int:
    args = _parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the sketched self-join of one workload is measured on a single "
              "MI355X (sharding across GPUs is not built)", file=sys.stderr)
        return 2
    import numpy as np
    import torch

    import datagen
    import paper_2311_03393_amd as skmp

    named_prec, named_refresh = NAMED[args.workload]
    prec = args.prec or named_prec
    refresh = args.refresh if args.refresh is not None else (named_refresh if prec == named_prec else 0)
    if args.join == "ab":
        return _bench_ab(args, prec, refresh)
    if args.stream:
        return _bench_stream(args, prec, refresh)
    if args.experiment == "random-walks":
        return _experiment_random_walks(args)

    dev = torch.device("cuda:0")
    if args.workload == "merchant-batch":
        w, T = datagen.make_merchant_batch_device(torch, dev)
    else:
        w = datagen.make(args.workload)
        T = torch.from_numpy(w.T).to(dev)
    d, N = T.shape
    k, m = w.k, w.m
    offsets = w.offsets
    n_series = len(offsets) - 1
    lens = np.diff(offsets)
    n_subs = lens - m + 1
    R = torch.empty((k, N), dtype=torch.float64, device=dev)
    stats = torch.empty((n_series, d, 2), dtype=torch.float64, device=dev)
    P = torch.empty((k, N), dtype=torch.float64, device=dev)
    I = torch.empty((k, N), dtype=torch.int64, device=dev)
    out = (torch.empty((n_series, 10), dtype=torch.int64, device=dev),
           torch.empty((n_series, 10), dtype=torch.int32, device=dev),
           torch.empty((n_series, 10), dtype=torch.float64, device=dev),
           torch.empty((n_series,), dtype=torch.int32, device=dev))
    # the large single-series workload also adds and removes dimensions and
    # recomputes the profile of the changed groups inside every step
    upd = w.update if args.workload == "large-series" else None
    joins = 2 if upd else 1
    if upd:
        T_add = torch.from_numpy(upd["T_add"]).to(dev)
        rem_ids = upd["rem_ids"]
        T_rem = T[torch.from_numpy(rem_ids).to(dev)].contiguous()
        rem_idx = torch.from_numpy(rem_ids).to(dev)
    cells = w.cells() * joins
    valid = k * sum(_valid_half_pairs(int(x), w.excl) for x in n_subs)  # per self-join launch
    # window columns (P and I are defined there only)
    wmask_h = np.zeros(N, dtype=bool)
    for a, ns in zip(offsets[:-1], n_subs):
        wmask_h[int(a):int(a) + int(ns)] = True
    wmask = torch.from_numpy(wmask_h).to(dev)
    profiles, picks, groups = {}, {}, {}

    def measure(pr: str, rf: int, steps: int, warmup: int):
        ws = torch.empty(skmp.mp_selfjoin_workspace(offsets, k, m, pr), dtype=torch.uint8, device=dev)

        def step():
            skmp.sketch_build(T, offsets, k, w.kind, w.sketch_seed, dim_ids=w.dim_ids, R=R, stats=stats)
            skmp.mp_selfjoin(R, offsets, k, m, w.excl, prec=pr, refresh=rf, P=P, I=I, workspace=ws)
            skmp.top_discords(P, offsets, k, m, 10, out=out)
            if upd:
                _, changed = skmp.sketch_update_dims(R, w.kind, k, w.sketch_seed, T_add=T_add,
                                                     add_ids=upd["add_ids"], T_rem=T_rem, rem_ids=rem_ids,
                                                     rem_stats=stats[0].index_select(0, rem_idx))
                skmp.mp_selfjoin(R, offsets, k, m, w.excl, prec=pr, refresh=rf, group_mask=changed, P=P, I=I,
                                 workspace=ws)
                skmp.top_discords(P, offsets, k, m, 10, out=out)

        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        _progress(f"{pr}: {warmup} warmup step(s) done")
        graph = None
        if not args.eager:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                step()
            torch.cuda.synchronize()
        skmp.timing_enable(True)
        for st in skmp.TIMERS:
            skmp.timing_read(st, reset=True)
        if graph is not None:  # stage timings from eager steps; the timed loop replays the graph
            for _ in range(steps):
                step()
            torch.cuda.synchronize()
            skmp.timing_enable(False)
        # every timed step is bracketed by events on the stream the library runs on (torch's current
        # stream): median and minimum per step beside the mean over the K steps
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for e0, e1 in evs:
            e0.record()
            if graph is not None:
                graph.replay()
            else:
                step()
            e1.record()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        per_step = sorted(e0.elapsed_time(e1) for e0, e1 in evs)
        _progress(f"{pr}: {steps} timed step(s), {(t1 - t0) * 1e3 / steps:.3f} ms each "
                  f"(median {per_step[len(per_step) // 2]:.3f}, min {per_step[0]:.3f})")
        skmp.timing_enable(False)
        stage = {st: skmp.timing_read(st, reset=True) for st in skmp.TIMERS}
        del ws, graph
        ms = (t1 - t0) * 1e3 / steps
        tiles_ms, tiles_n = stage["tiles"]
        tile_avg_s = tiles_ms / max(tiles_n, 1) * 1e-3
        profiles[pr] = P[:, wmask].clone()
        picks[pr] = out[0].cpu().clone()
        groups[pr] = out[1].cpu().clone()
        med = float(np.median(per_step))
        return {
            "precision": pr, "refresh": rf, "ms_per_step": ms, "cells_per_s": cells / (ms * 1e-3),
            "ms_per_step_median": med, "ms_per_step_min": per_step[0], "cells_per_s_median": cells / (med * 1e-3),
            "tile_kernel_ms": tile_avg_s * 1e3, "tile_launches": tiles_n,
            "tile_frac_of_vector_peak": (OPS_PER_CELL * valid / tile_avg_s / PUBLISHED_PEAK[pr]
                                         if pr in PUBLISHED_PEAK else None),
            "tile_frac_of_issue_model": (valid / tile_avg_s / CELL_PEAK[pr] if pr in CELL_PEAK else None),
            "tile_frac_of_mfma_peak": (_mfma_flops_per_cell(_mixed_form(rf), m) * valid / tile_avg_s / MFMA_16BIT_PEAK
                                       if pr in ("bf16x3", "fp16x3") else None),
            "form": _mixed_form(rf) if pr in ("bf16x3", "fp16x3") else "diagonal",
            "stages_ms_per_step": {st: v[0] / max(steps, 1) for st, v in stage.items()},
            "top10": [int(x) for x in out[0][0].cpu()],
        }

    if args.copy_calib > 0:
        src = torch.empty(args.copy_calib << 20, dtype=torch.uint8, device=dev).fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    tuned = {}
    if args.autotune:
        skmp.sketch_build(T, offsets, k, w.kind, w.sketch_seed, dim_ids=w.dim_ids, R=R, stats=stats)
        sub = np.arange(n_series) if n_series <= 64 else np.sort(np.random.default_rng(2).choice(n_series, 64, False))
        if n_series > 64:  # a representative subset: its own concatenation of the chosen series
            cols = np.concatenate([np.arange(offsets[s], offsets[s + 1]) for s in sub])
            R_t = R[:, torch.from_numpy(cols).to(dev)].contiguous()
            offs_t = np.concatenate([[0], np.cumsum(lens[sub])])
        else:
            R_t, offs_t = R, offsets
        for pr in sorted({prec, "fp64"} & {"fp64", "fp32"}):
            tuned[pr] = skmp.mp_selfjoin_autotune(R_t, offs_t, k, m, w.excl, prec=pr,
                                                  refresh=refresh if pr == prec else 0, reps=1)
        del R_t
        torch.cuda.synchronize()
    also = args.also
    if also is None:
        also = "fp64" if args.workload in ("merchant-batch", "large-series") else "fp64,fp32,bf16x3,fp16x3"
    head = measure(prec, refresh, args.steps, args.warmup)
    paths = {f"{prec}" + (f"_refresh{refresh}" if refresh else ""): head}
    for extra in [x for x in also.split(",") if x and x != prec]:
        paths[extra] = measure(extra, 0, max(3, args.steps // 2), 1)
    if "fp64" in profiles:
        # error of every path against the FP64 path (itself held to the oracle at 1e-9 * 2 sqrt(m))
        ref = profiles["fp64"]
        tol = 1e-3 * 2 * m ** 0.5
        for key, v in paths.items():
            got = profiles[v["precision"]]
            both = torch.isfinite(ref) & torch.isfinite(got)
            err = (got - ref).abs()[both]
            sq = (got * got - ref * ref).abs()[both]
            v["vs_fp64"] = {
                "max_abs_dP": float(err.max()) if err.numel() else 0.0,
                "max_abs_dP2": float(sq.max()) if sq.numel() else 0.0,
                "finite_pattern_equal": bool(torch.equal(torch.isfinite(ref), torch.isfinite(got))),
                "tolerance_dP": tol,
                "top10_equal_all_series": bool(torch.equal(picks[v["precision"]], picks["fp64"])),
                "series_with_different_top10": int((picks[v["precision"]] != picks["fp64"]).any(dim=1).sum()),
            }
            del got, both, err, sq
        del ref
    profiles.clear()

    # discord dimension detection (Algorithm 3) for the named path's top discord:
    # all dimensions of its group, self-join setting, FP64
    dimdet = None
    if n_series == 1 and not args.no_dims:
        i_star, g_star = int(picks[prec][0, 0]), int(groups[prec][0, 0])
        if i_star >= 0 and g_star >= 0:
            dims = skmp.group_dims(w.kind, k, w.sketch_seed, g_star, w.dim_ids)
            skmp.dim_detect(T, stats[0], dims, i_star, m, excl=w.excl)   # warm-up
            torch.cuda.synchronize()
            skmp.timing_enable(True)
            skmp.timing_read("dimdetect", reset=True)
            reps = 5
            for _ in range(reps):
                sc, nn_, best = skmp.dim_detect(T, stats[0], dims, i_star, m, excl=w.excl)
            torch.cuda.synchronize()
            skmp.timing_enable(False)
            dd_ms, dd_n = skmp.timing_read("dimdetect", reset=True)
            per = dd_ms / max(dd_n, 1)
            n_sub0 = int(lens[0]) - m + 1
            ops = float(len(dims)) * n_sub0 * 7.0 * m   # mean, variance and distance passes, FP64
            dimdet = {"i_star": i_star, "group": g_star, "n_dims": int(len(dims)),
                      "j_star": int(dims[int(best.item())]), "ms": per,
                      "roofline": {"bound": "alu", "achieved": ops / (per * 1e-3) / 1e12,
                                   "peak": PUBLISHED_PEAK["fp64"] / 1e12, "unit": "TFLOP/s",
                                   "frac": ops / (per * 1e-3) / PUBLISHED_PEAK["fp64"],
                                   "basis": "7 m FP64 operations per (dimension, train subsequence) counted as "
                                            "flops (mean, variance, explicit-difference distance), against the "
                                            "published FP64 vector peak 78.6 TFLOP/s"}}

    tile_avg_s = head["tile_kernel_ms"] * 1e-3
    tr = _traffic(KERNELS[prec], args.workload)
    if prec in ("bf16x3", "fp16x3"):
        # products on the matrix cores: three 16-bit products (hi*hi, hi*lo, lo*hi) per valid cell, of
        # depth 32 per 16-row tile step (blocked) or m (Hankel-direct), 2 flops per multiply-add
        form = _mixed_form(refresh)
        fpc = _mfma_flops_per_cell(form, m)
        achieved = fpc * valid / tile_avg_s
        kern = KERNELS[prec] if form == "blocked" else KERNELS_HANKEL[prec]
        roofline = {
            "bound": "mfma",
            "achieved": achieved / 1e12,
            "peak": MFMA_16BIT_PEAK / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / MFMA_16BIT_PEAK,
            "traffic": (tr["fetch_bytes"] + tr["write_bytes"]) if tr else None,
            "traffic_detail": tr,
            "kernel": kern,
            "form": form,
            "per_launch": {"cells": valid, "flops_per_cell": fpc, "avg_ms": head["tile_kernel_ms"],
                           "launches": head["tile_launches"]},
            "basis": f"dense 16-bit MFMA peak 2.5 PFLOP/s; {fpc:.0f} MFMA flops per valid half-matrix cell "
                     f"({'3 products of depth 32 per 16 x 16 tile step' if form == 'blocked' else '3 products of depth m'})",
            "vector_side": {"flops_per_cell": OPS_PER_CELL, "frac_of_fp32_peak":
                            OPS_PER_CELL * valid / tile_avg_s / PUBLISHED_PEAK["fp32"],
                            "basis": "the method's 6 operations per cell against the FP32 vector peak (the "
                                     "normalisation, keys and minima run on the VALU)"},
        }
    else:
        roofline = _roofline_vector(prec, valid, head["tile_kernel_ms"], head["tile_launches"], KERNELS[prec], tr)
    # the sketch stage is HBM-bound: T is read twice (statistics, projection), R written once
    sk_ms = head["stages_ms_per_step"]["sketch"]
    sk_bytes = 2.0 * d * N * T.element_size() + k * N * 8.0
    sketch = {"ms_per_step": sk_ms, "bytes": sk_bytes,
              "GB_per_s": sk_bytes / (sk_ms * 1e-3) / 1e9 if sk_ms > 0 else None,
              "frac_of_hbm": sk_bytes / (sk_ms * 1e-3) / 8e12 if sk_ms > 0 else None,
              "basis": "2 reads of T + 1 write of R against 8 TB/s"}
    if upd:
        sketch["note"] = "ms_per_step also holds the update's dimension statistics and projections"
    result = {
        "metric": "matrix-profile cells/sec (k*n^2/2 per s)",
        "value": head["cells_per_s"],
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "ms_per_step_median": head["ms_per_step_median"],
        "ms_per_step_min": head["ms_per_step_min"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32"}.get(prec, prec),
        "data": "synthetic",
        "graph": not args.eager,
        "autotuned": tuned or None,
        "config": {"workload": DESCR[args.workload] + (" + add/remove 16 dims and recompute" if upd else ""),
                   "precision": prec, "refresh": refresh, "self_joins_per_step": joins,
                   "n_series": n_series, "cells_per_step": cells, "valid_half_pairs_per_join": valid,
                   "parallelism": "single GPU"},
        "roofline": roofline,
        "sketch": sketch,
        "dim_detect": dimdet,
        "paths": paths,
    }
    if not args.no_cpu_baseline:
        rng = np.random.default_rng(1)
        pick = rng.choice(n_series, size=min(n_series, 8), replace=False)
        series = [(int(s), R[:, int(offsets[s]):int(offsets[s + 1])].cpu().numpy()) for s in pick]
        result["cpu_baseline"] = _cpu_baseline(series, w, args.cpu_seconds, full=args.cpu_full)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
