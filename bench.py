"""Benchmark: joined points/s of the ACT probe on one MI355X.

Workload (the paper's neighbourhood-scale join, synthetic stand-in): 290
Voronoi polygons over the NYC box (20..800 vertices, 5% with a hole) and
1e8 fp64 (lat, lng) points from a 64-component Gaussian mixture + 10%
uniform, resident in HBM before timing. One step = one act_join of all 1e8
points in exact mode (projection, trie descent, refinement, output); the
approximate mode at 4 m is timed the same way and reported beside it.

Prints one JSON line. `--gpus N` with N > 1 exits: this build targets one
GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_POINT = 20  # 16 B fp64 (lat, lng) in + 4 B int32 id out


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def time_joins(idx, pts, out, steps, warmup, refine=0):
    import torch
    for _ in range(warmup):
        idx.join_ex(pts, out, refine=refine)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        idx.join_ex(pts, out, refine=refine)
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms = [a.elapsed_time(b) for a, b in ev]
    return wall, kms


def cpu_baseline(P, workload, n_sample):
    import oracle
    import synth
    pts = synth.workload_points(workload, 0, n_sample)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    oracle.join(P, pts[:1000], nthreads=cores)
    t0 = time.perf_counter()
    oracle.join(P, pts, nthreads=cores)
    dt = time.perf_counter() - t0
    return {"value": n_sample / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": "first %d points of the %s stream, exact join (brute force, bbox "
                      "prefilter + exact PIP), %d threads, %.1f s" % (n_sample, workload, cores, dt)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2")
    ap.add_argument("--points", type=int, default=0, help="override the point count")
    ap.add_argument("--cpu-sample", type=int, default=4_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-approx", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the probe replicates the immutable index per GPU and "
              "splits points, and this build runs and reports the single-GPU case only "
              "(--gpus %d refused)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1802_09488_amd as act

    w = synth.WORKLOADS[args.workload]
    n = args.points or w["n_points"]
    log("polygons", args.workload)
    P = synth.workload_polygons(args.workload)
    t0 = time.perf_counter()
    idx = act.build(P, "exact")
    t_build_exact = time.perf_counter() - t0
    idx_a = None
    if not args.no_approx:
        t0 = time.perf_counter()
        idx_a = act.build(P, "approx", 4.0)
        t_build_approx = time.perf_counter() - t0
    log("generating %d points" % n)
    pts = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    step = 1 << 24
    for s in range(0, n, step):
        e = min(n, s + step)
        pts[s:e].copy_(torch.from_numpy(synth.workload_points(args.workload, s, e)))
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()

    log("timing exact")
    wall, kms = time_joins(idx, pts, out, args.steps, args.warmup)
    kernel_ms = float(np.mean(kms))
    ms_per_step = 1000.0 * wall / args.steps
    value = n * args.steps / wall
    _, _, ctr = idx.join_ex(pts, out, counters=True)
    wall64, kms64 = time_joins(idx, pts, out, max(3, args.steps // 2), 1,
                               refine=act.ACT_REFINE_FP64)
    res = {
        "metric": "joined points/sec (exact & approx@4m) + HBM roofline %; p50/p99 batch latency",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %d Voronoi polygons (NYC box), %d fp64 mixture points, "
                               "exact join (covering level 20); approx@4m beside it"
                               % (args.workload, P.n_polys, n),
                   "n_points": n, "n_polys": P.n_polys, "n_edges": int(idx.stats()["n_edges"]),
                   "mode": "exact", "parallelism": "single GPU"},
    }
    achieved = BYTES_PER_POINT * n / (kernel_ms * 1e-3) / 1e9
    res["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS,
                       "unit": "GB/s", "frac": achieved / PEAK_HBM_GBS, "traffic": None,
                       "kernel": "probe_kernel", "kernel_ms": kernel_ms,
                       "bytes_per_point": BYTES_PER_POINT}
    res["fp32_filter_vs_fp64"] = {"fp32_filter_points_per_s": value,
                                  "fp64_points_per_s": n * len(kms64) / wall64,
                                  "fp64_kernel_ms": float(np.mean(kms64))}
    res["counters"] = ctr
    st = idx.stats()
    res["index"] = {"exact": {k: st[k] for k in ("n_cells", "n_nodes", "node_bytes", "lut_words",
                                                 "device_bytes", "max_depth")},
                    "build_s_exact": t_build_exact}
    if idx_a is not None:
        log("timing approx@4m")
        wa, kma = time_joins(idx_a, pts, out, args.steps, args.warmup)
        sa = idx_a.stats()
        res["approx4m"] = {"points_per_s": n * args.steps / wa, "kernel_ms": float(np.mean(kma)),
                           "hbm_frac": BYTES_PER_POINT * n / (np.mean(kma) * 1e-3) / 1e9
                           / PEAK_HBM_GBS}
        res["index"]["approx4m"] = {k: sa[k] for k in ("n_cells", "n_nodes", "node_bytes",
                                                       "device_bytes", "max_depth")}
        res["index"]["build_s_approx4m"] = t_build_approx
    del pts, out
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline")
        res["cpu_baseline"] = cpu_baseline(P, args.workload, min(args.cpu_sample, n))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
