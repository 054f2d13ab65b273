"""Benchmark: joined points/s of the ACT probe on one MI355X.

Workload (the paper's neighbourhood-scale join, synthetic stand-in): 290
Voronoi polygons over the NYC box (20..800 vertices, 5% with a hole) and
1e8 fp64 (lat, lng) points from a 64-component Gaussian mixture + 10%
uniform, resident in HBM before timing. One step = one act_join of all 1e8
points in exact mode (projection, trie descent, candidate resolution with
exact refinement, output). Reported beside it: the approximate mode at 4 m,
the refinement variants (cell-local, fp32 filter + fp64/exact re-test over
all edges, all-fp64 over all edges), per-step latency percentiles, the
probe kernel's HBM roofline, and the CPU oracle on the host's cores.

Prints one JSON line. `--gpus N` with N > 1 exits: the run measures one GPU.

Profile helpers (turn rocprofv3 output of a run of this script into the
text summaries kept under profiles/):
  python bench.py --summarize-trace DIR      (rocprofv3 --kernel-trace --stats
                                              --output-format csv -d DIR)
  python bench.py --summarize-pmc FDIR WDIR  (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
                                              --output-format csv -d FDIR / WDIR)
  python bench.py --summarize-counters [--points-per-launch N] DIR...
                                             (rocprofv3 --pmc <SQ_/TCC_ counters>
                                              --output-format csv -d DIR, one per set)
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0
BYTES_PER_POINT = 20  # 16 B fp64 (lat, lng) in + 4 B int32 id out
# Finest covering level of the benchmarks' exact indexes: 22 fills the
# deepest trie node level (levels 19-22 under the workloads' prefix level 6)
# and halves the candidate cells per level over the library's default of 20
# without another node level (c3: 0.66 -> 0.41 ms per 2^24 points).
EXACT_LEVEL = 22
COPY_BYTES = 1 << 30  # calibration copy (device to device)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_probe_c2.md")
KERNEL_SOURCES = ["probe.hip", "geom.hpp", "cellid.hpp", "index.hpp"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


HOST_SIDE_MARKER = b"// ============================================== host side"


def kernel_source_hash() -> str:
    """sha256 (first 16 hex digits) of the device code: probe.hip up to its
    host-side marker (kernels and device functions; the launches and the C
    ABI after it do not change what a kernel does) and the headers the
    kernels include."""
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1802_09488_amd", "csrc", f), "rb") as fh:
            b = fh.read()
        if f == "probe.hip":
            k = b.find(HOST_SIDE_MARKER)
            if k < 0:
                raise SystemExit("probe.hip has no host-side marker")
            b = b[:k]
        h.update(b)
    return h.hexdigest()[:16]


COUNTERS_FILE = os.path.join(ROOT, "profiles", "probe_counters_c2.md")
# VALU issue ceiling: 1024 SIMDs x 2.4 GHz, one 64-lane wave instruction
# every 4 cycles per SIMD (fp64 FMA at full rate), in lane operations/s
PEAK_VALU_LANE_OPS = 1024 * 2.4e9 / 4 * 64


def measured_valu():
    """VALU instructions per 64 points of the probe kernels, from the
    committed counter summary, if it was taken on the current kernel
    sources (else None)."""
    if not os.path.exists(COUNTERS_FILE):
        return None
    txt = open(COUNTERS_FILE).read()
    m = re.search(r"kernel sources sha256/16: `([0-9a-f]+)`", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    out = {}
    for mode, label in (("approx", "0"), ("exact", "3")):
        r = re.search(r"\| probe_kernel<%s, 2, 0, 2, false, false> \| \d+ \| ([0-9.e+]+) \|" % label,
                      txt)
        if r:
            out[mode] = float(r.group(1))
    return out or None


def measured_traffic():
    """Probe HBM bytes per launch from the committed counter summary, if it
    was taken on the current kernel sources (else None)."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    txt = open(TRAFFIC_FILE).read()
    m = re.search(r"kernel sources sha256/16: `([0-9a-f]+)`", txt)
    if not m or m.group(1) != kernel_source_hash():
        return None
    out = {}
    for mode in ("exact", "approx"):
        r = re.search(r"\| probe_kernel %s \| ([0-9.e+]+) \|" % mode, txt)
        if r:
            out[mode] = float(r.group(1))
    return out or None


def percentile(v, q):
    import numpy as np
    return float(np.percentile(np.asarray(v), q))


def time_joins(idx, pts, out, steps, warmup, **kw):
    """Times `steps` joins (after `warmup`): wall clock around `steps`
    back-to-back joins with nothing else on the stream; then, in a second
    pass of `steps` joins outside that window, HIP events around each join
    and after its probe kernel (event records between the launches would
    otherwise add their own gaps to the wall-clock figure)."""
    import torch
    for _ in range(warmup):
        idx.join_ex(pts, out, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        idx.join_ex(pts, out, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = [tuple(torch.cuda.Event(enable_timing=True) for _ in range(3)) for _ in range(steps)]
    for _, m, _ in ev:
        m.record()  # creates the event the library records after the probe
    torch.cuda.synchronize()
    for a, m, b in ev:
        a.record()
        idx.join_ex(pts, out, probe_event=m, **kw)
        b.record()
    torch.cuda.synchronize()
    total = [a.elapsed_time(b) for a, _, b in ev]
    probe = [a.elapsed_time(m) for a, m, _ in ev]
    return wall, total, probe


def copy_calibration():
    """A plain device-to-device copy of COPY_BYTES (the hipMemcpy blit
    kernel): its rocprofv3 FETCH_SIZE / WRITE_SIZE readings calibrate the
    counters, and its rate is the achievable copy bandwidth."""
    import torch
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b)
    del src, dst
    return {"bytes_each_way": COPY_BYTES, "ms": ms, "GBps_read_plus_write": 2 * COPY_BYTES / ms / 1e6}


def batched_leg(act, idx, pts, exact_out, seed=3004, hi=1e6, replays=5):
    """The resident points cut into uneven batches (sizes floor(exp(U(0,
    ln 1e6)))), joined by one batched join captured in a HIP graph and
    replayed: throughput, the replay's duration, and per-batch completion
    latency (GPU wall-clock ticks from the join's start)."""
    import numpy as np
    import torch
    n = pts.shape[0]
    g = np.random.default_rng(seed)
    sizes = []
    tot = 0
    while tot < n:
        k = int(min(n - tot, max(1, np.floor(np.exp(g.uniform(0.0, np.log(hi)))))))
        sizes.append(k)
        tot += k
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    batches = [(pts[a:b], out[a:b]) for a, b in zip(bounds[:-1], bounds[1:])]
    desc, total = act.batch_descriptors(batches)
    ticks = torch.zeros(len(batches) + 1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    idx.batched_reserve(len(batches), total, stream=s)
    with torch.cuda.stream(s):
        idx.join_batched(desc, total, ticks=ticks)  # eager once (warm)
    s.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        idx.join_batched(desc, total, ticks=ticks)
    hz = act.wall_clock_hz(0)
    ms, lat50, lat99 = [], [], []
    for _ in range(replays):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        a.record()
        graph.replay()
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
        t = ticks.cpu().numpy().view(np.uint64).astype(np.float64)
        lat = (t[1:] - t[0]) / hz * 1e3
        lat50.append(float(np.percentile(lat, 50)))
        lat99.append(float(np.percentile(lat, 99)))
    ok = bool(np.array_equal(out.cpu().numpy(), exact_out)) if exact_out is not None else None
    return {"batches": len(batches), "points": int(total),
            "batch_sizes": "floor(exp(U(0, ln 1e6))), seed %d" % seed,
            "graph_replay_ms": float(np.median(ms)),
            "points_per_s": total / (float(np.median(ms)) * 1e-3),
            "batch_latency_ms": {"p50": float(np.median(lat50)), "p99": float(np.median(lat99)),
                                 "what": "per-batch completion tick minus the join's start "
                                         "tick (GPU wall clock), one graph replay"},
            "identical_to_single_join": ok}


def serving_leg(act, indexes, pools, qps_list, seconds, seed=5005, slots=8,
                arena_bytes=2 << 30, max_points=65536):
    """Serving: requests of floor(exp(U(0, ln 65536))) points, each aimed at
    one of the resident indexes (Bernoulli 1/2), arriving as a Poisson
    process at each rate in qps_list for `seconds`; points are windows of
    the indexes' point pools (host). The requests are replayed by the
    library's native load generator (act_server_replay: one thread paces the
    submissions on the server's clock, another waits for completions).
    Latency = completion (results in host memory) minus scheduled arrival."""
    import numpy as np
    # requests are at most max_points long; a launch group joins up to 2^20
    srv = act.Server(indexes, slots=slots, arena_bytes=arena_bytes, max_request_points=1 << 20)
    g = np.random.default_rng(seed)
    pools = [np.ascontiguousarray(q, dtype=np.float64) for q in pools]
    ptrs = [q.ctypes.data for q in pools]
    res = []
    for qps in qps_list:
        nreq = int(qps * seconds)
        sizes = np.floor(np.exp(g.uniform(0.0, np.log(max_points), nreq))).astype(np.int64)
        target = g.integers(0, len(indexes), nreq)
        gaps = g.exponential(1.0 / qps, nreq)
        room = np.array([len(q) for q in pools], dtype=np.int64)[target] - sizes
        starts = (g.random(nreq) * room).astype(np.int64)
        # the replay allocates and writes its output ring before its first
        # submission: the first arrival is far enough ahead for that
        arrival = act.Server.clock() + 0.25 + np.cumsum(gaps)
        tm = srv.replay(target, ptrs, starts, sizes, arrival)
        lat = tm["done_s"] - tm["arrival_s"]
        queued = tm["admitted_s"] - tm["arrival_s"]  # waiting for a slot and memory
        phases = {"staging": tm["launched_s"] - tm["admitted_s"],   # points into pinned memory
                  "gpu": tm["results_s"] - tm["launched_s"],        # copies and join, found done
                  "copy_out": tm["done_s"] - tm["results_s"]}       # results to the callers
        span = float(np.max(tm["done_s"]) - arrival[0]) if nreq else 1.0
        res.append({"qps_offered": qps, "requests": nreq, "seconds": seconds,
                    "points": int(sizes.sum()), "points_per_s": float(sizes.sum()) / span,
                    "latency_ms": {"p50": 1e3 * float(np.percentile(lat, 50)),
                                   "p99": 1e3 * float(np.percentile(lat, 99)),
                                   "max": 1e3 * float(np.max(lat))},
                    "queued_ms": {"p50": 1e3 * float(np.percentile(queued, 50)),
                                  "p99": 1e3 * float(np.percentile(queued, 99))},
                    "service_p99_ms": {k: 1e3 * float(np.percentile(v, 99))
                                       for k, v in phases.items()},
                    "slowest_request_ms": {k: 1e3 * float(v[int(np.argmax(lat))])
                                           for k, v in dict(phases, queued=queued).items()},
                    "qps_achieved": nreq / span})
    st = srv.stats()
    srv.close()
    return {"slots": slots, "arena_bytes": int(arena_bytes), "load_generator": "act_server_replay",
            "request_points": "floor(exp(U(0, ln %d))), seed %d" % (max_points, seed),
            "runs": res, "failed": st["failed"], "requests": st["completed"],
            "launch_groups": st["launches"],
            "scheduler_max_ms": {"pass": 1e3 * st["max_pass_s"], "launch": 1e3 * st["max_launch_s"],
                                 "stage": 1e3 * st["max_stage_s"],
                                 "finish": 1e3 * st["max_finish_s"]}}


def cpu_baseline_and_parity(P, workload, n_sample, gpu_out, gpu_pairs=None, gpu_counts=None,
                            one_thread_points=1_000_000):
    """The oracle (brute force: bbox prefilter + exact point-in-polygon
    against every polygon, OpenMP over points) on the host's cores over the
    first n_sample points of the stream; its output is compared with the
    GPU's exact-mode output for those points: out[], and, when given, the
    GPU's further (point, polygon) pairs and per-polygon counts. The oracle
    is also timed on one thread over the first one_thread_points points."""
    import numpy as np

    import oracle
    import synth
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    oracle.join(P, synth.workload_points(workload, 0, 1000), nthreads=cores)  # warm
    step = 1 << 24
    dt = 0.0
    mism = 0
    ref_pairs = []
    counts = np.zeros(P.n_polys, np.int64)
    for s in range(0, n_sample, step):
        e = min(n_sample, s + step)
        pts = synth.workload_points(workload, s, e)
        t0 = time.perf_counter()
        ref = oracle.join(P, pts, nthreads=cores)
        dt += time.perf_counter() - t0
        mism += int(np.count_nonzero(ref.out != gpu_out[s:e]))
        if len(ref.pairs):
            ref_pairs.append(ref.pairs + np.array([s, 0]))
        counts += np.bincount(ref.pair_set()[:, 1], minlength=P.n_polys)
    base = {"value": n_sample / dt, "unit": "points/s", "cores": cores, "kind": "oracle",
            "sample": "points 0..%d of the %s stream (%s), exact join, %d threads, %.1f s"
                      % (n_sample, workload, "the whole workload" if n_sample == len(gpu_out)
                         else "a prefix", cores, dt)}
    n1 = min(one_thread_points, n_sample)
    pts = synth.workload_points(workload, 0, n1)
    t0 = time.perf_counter()
    oracle.join(P, pts, nthreads=1)
    d1 = time.perf_counter() - t0
    base["one_thread"] = {"value": n1 / d1, "unit": "points/s", "cores": 1,
                          "sample": "points 0..%d of the %s stream, exact join, 1 thread, %.1f s"
                                    % (n1, workload, d1)}
    parity = {"points_checked": n_sample, "out_mismatches": mism}
    if gpu_pairs is not None:
        rp = np.concatenate(ref_pairs) if ref_pairs else np.zeros((0, 2), np.int64)
        rp = rp[np.lexsort((rp[:, 1], rp[:, 0]))]
        gp = gpu_pairs[(gpu_pairs[:, 0] < n_sample)]
        gp = gp[np.lexsort((gp[:, 1], gp[:, 0]))]
        parity["pairs_checked"] = int(len(rp))
        parity["pairs_identical"] = bool(np.array_equal(rp, gp))
    if gpu_counts is not None and n_sample == len(gpu_out):
        parity["counts_identical"] = bool(np.array_equal(counts, gpu_counts))
        parity["count_pairs_total"] = int(counts.sum())
    return base, parity


def paper_config_leg(act, P, workload, pts, out, steps, n_train=1_000_000):
    """The paper's covering configuration (Section V: per-polygon coverings of
    at most 128 cells up to level 30 and 256 interior cells up to level 20,
    merged), untrained and trained with n_train points of the workload's
    distribution (Section III-D): exact-join time on the resident points and
    the index metrics of the paper's Tables III and IV (tree nodes, false
    hits, solely true hits, candidates per refined point)."""
    import numpy as np
    import synth
    n = pts.shape[0]
    res = {"covering": "max covering cells 128, max level 30, max interior cells 256, "
                       "max interior level 20", "n_train": n_train}
    for name, tp in (("untrained", None), ("trained", synth.training_points(workload, n_train))):
        t0 = time.perf_counter()
        ix = act.build(P, "exact", max_level=30, max_covering_cells=128, train_points=tp)
        tb = time.perf_counter() - t0
        ix.reserve(n)
        wall, tot, _ = time_joins(ix, pts, out, steps, 1)
        _, _, ctr = ix.join_ex(pts, out, counters=True)
        st = ix.stats()
        res[name] = dict(_index_metrics(ctr), tree_nodes=st["n_nodes"], cells=st["n_cells"],
                         image_bytes=st["image_bytes"], train_splits=st["train_splits"],
                         build_s=tb, join_ms_mean=float(np.mean(tot)),
                         points_per_s=n * steps / wall)
        del ix
    return res


def precomputed_ids_leg(act, indexes, pts, steps, exact_out):
    """Joins of points that arrive with their level-30 cell ids (the paper's
    probe input): the ids are computed once (act_cell_ids, timed too), then
    act_join_ids is timed per index; its algorithmic traffic is 12 B per
    point (8 B id in, 4 B id out) plus 16 B per pending point in exact
    mode."""
    import numpy as np
    import torch
    n = pts.shape[0]
    ids = torch.empty(n, dtype=torch.int64, device="cuda")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    ms = []
    for k in range(steps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        act.cell_ids(pts, out=ids)
        b.record()
        torch.cuda.synchronize()
        if k:
            ms.append(a.elapsed_time(b))
    res = {"cell_ids_ms_median": float(np.median(ms))}
    for name, idx in indexes:
        exact = idx.mode == act.ACT_EXACT
        ms = []
        for k in range(steps + 1):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            idx.join_ids(ids, pts if exact else None, out=out)
            b.record()
            torch.cuda.synchronize()
            if k:
                ms.append(a.elapsed_time(b))
        med = float(np.median(ms))
        r = {"join_ms_median": med, "points_per_s": n / (med * 1e-3),
             "roofline_frac_12B": 12 * n / (med * 1e-3) / 1e9 / PEAK_HBM_GBS}
        if exact:
            r["identical_to_join"] = bool(np.array_equal(out.cpu().numpy(), exact_out))
        res[name] = r
    del ids, out
    return res


def pairs_and_counts_leg(act, indexes, pts, steps):
    """Timed pair-emitting joins (act_join_pairs: out[] plus every further
    (point, polygon) pair) and per-polygon count joins (act_join_count) over
    the resident points, for each (name, index); buffers are allocated once
    and the counters zeroed before each timed call. Returns the timings and
    the exact index's pairs and counts (host) for the oracle check."""
    import ctypes

    import numpy as np
    import torch
    n = pts.shape[0]
    lib = act.lib
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    cap = n // 8
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    pp = torch.empty(cap, dtype=torch.int64, device="cuda")
    pq = torch.empty(cap, dtype=torch.int32, device="cuda")
    npairs = torch.zeros(1, dtype=torch.int64, device="cuda")
    P_ = ctypes.c_void_p
    res, keep = {}, {}
    for name, idx in indexes:
        npoly = idx.n_polys
        counts = torch.zeros(npoly, dtype=torch.int64, device="cuda")

        def pairs_call():
            act._b.check(lib.act_join_pairs(idx.handle, P_(pts.data_ptr()), n, P_(out.data_ptr()),
                                            P_(pp.data_ptr()), P_(pq.data_ptr()), cap,
                                            P_(npairs.data_ptr()), st))

        def count_call():
            act._b.check(lib.act_join_count(idx.handle, P_(pts.data_ptr()), n,
                                            P_(counts.data_ptr()), st))
        r = {}
        for what, call, zero in (("pairs", pairs_call, npairs), ("count", count_call, counts)):
            ms = []
            for k in range(steps + 1):
                zero.zero_()
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record()
                call()
                b.record()
                torch.cuda.synchronize()
                if k:
                    ms.append(a.elapsed_time(b))
            med = float(np.median(ms))
            r[what] = {"join_ms_median": med, "points_per_s": n / (med * 1e-3)}
        m = int(npairs.item())
        r["pairs"]["extra_pairs"] = m
        r["pairs"]["complete"] = m <= cap
        r["count"]["pairs_counted"] = int(counts.sum().item())
        res[name] = r
        if name == "exact":
            keep["pairs"] = torch.stack([pp[:min(m, cap)],
                                         pq[:min(m, cap)].to(torch.int64)], 1).cpu().numpy()
            keep["counts"] = counts.cpu().numpy()
    del out, pp, pq
    return res, keep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="all", choices=["all", "c2", "c3", "c4", "c5"],
                    help="all (default): the c2 headline (290 polygons, 1e8 points) plus "
                         "compact c3/c4/c5 legs; c2: the headline alone; c3: 40k polygons, "
                         "1e9 points in 2^24 batches; c4: 10,000 uneven batches, one graph "
                         "replay; c5: serving sweep")
    ap.add_argument("--points", type=int, default=0, help="override the point count")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="oracle points (default: the whole c2 workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile", action="store_true",
                    help="c2: only the headline exact and approx@4m joins (for rocprofv3 runs)")
    ap.add_argument("--serve-seconds", type=float, default=0.0,
                    help="seconds per serving rate (default 2 in c2, 4 in c5)")
    ap.add_argument("--summarize-trace", metavar="DIR")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"))
    ap.add_argument("--summarize-counters", nargs="+", metavar="DIR")
    ap.add_argument("--points-per-launch", type=float, default=0.0,
                    help="with --summarize-counters: points one launch processes")
    args = ap.parse_args()
    if args.summarize_trace:
        return summarize_trace(args.summarize_trace)
    if args.summarize_pmc:
        return summarize_pmc(*args.summarize_pmc)
    if args.summarize_counters:
        return summarize_counters(args.summarize_counters, args.points_per_launch)
    if args.gpus != 1:
        print("bench.py measures one GPU: the probe replicates the immutable index per GPU and "
              "splits the points, and this benchmark runs and reports the single-GPU case only "
              "(--gpus %d refused)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    {"all": run_all, "c2": run_c2, "c3": run_c3, "c4": run_c4, "c5": run_c5}[args.workload](args)


def run_all(args):
    """The c2 headline line, with compact c3, c4 and c5 legs in it."""
    res, keep = run_c2(args, emit=False)
    if res is None:
        return
    res["legs"] = compact_legs(args, keep)
    print(json.dumps(res), flush=True)


def run_c2(args, emit=True):
    import numpy as np
    import torch

    import synth
    import paper_1802_09488_amd as act

    args.workload = "c2"
    w = synth.WORKLOADS[args.workload]
    n = args.points or w["n_points"]
    log("polygons", args.workload)
    P = synth.workload_polygons(args.workload)
    t0 = time.perf_counter()
    idx = act.build(P, "exact", max_level=EXACT_LEVEL)
    t_build_exact = time.perf_counter() - t0
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
    idx.reserve(n)  # one pass over all points
    torch.cuda.synchronize()
    calib = copy_calibration()
    tuned = None
    if not args.profile:
        # the autotuner's pick on this GPU, on separate copies of the indexes:
        # the timed joins below use the default launch configuration, the one
        # the committed kernel profiles were taken with
        # tuned on the whole workload: a smaller sample favours smaller grids
        log("autotuner on all points")
        tuned = {"exact": act.build(P, "exact", max_level=EXACT_LEVEL).tune(pts),
                 "approx4m": act.build(P, "approx", 4.0).tune(pts)}

    log("timing exact")
    wall, tot, prb = time_joins(idx, pts, out, args.steps, args.warmup)
    value = n * args.steps / wall
    exact_out = out.cpu().numpy()
    _, _, ctr = idx.join_ex(pts, out, counters=True)
    log("timing approx@4m")
    wall_a, tot_a, prb_a = time_joins(idx_a, pts, out, args.steps, args.warmup)
    _, _, ctr_a = idx_a.join_ex(pts, out, counters=True)
    if args.profile:
        res = {"profile_run": True, "exact_probe_ms": float(np.mean(prb)),
               "approx_probe_ms": float(np.mean(prb_a)),
               "kernel_sources_sha256_16": kernel_source_hash()}
        print(json.dumps(res), flush=True)
        return None, None
    log("timing refinement variants")
    k = max(3, args.steps // 2)
    var = {}
    for name, mode in (("local", act.ACT_REFINE_LOCAL), ("fp32_filter", act.ACT_REFINE_FP32_FILTER),
                       ("fp64", act.ACT_REFINE_FP64)):
        wv, tv, pv = time_joins(idx, pts, out, k, 1, refine=mode)
        var[name] = {"points_per_s": n * k / wv, "join_ms_mean": float(np.mean(tv)),
                     "resolve_ms_mean": float(np.mean(tv) - np.mean(pv))}
        if mode != act.ACT_REFINE_LOCAL:
            torch.cuda.synchronize()
            var[name]["identical_to_local"] = bool(np.array_equal(out.cpu().numpy(), exact_out))
    var["fp32_filter_over_fp64_speedup"] = (var["fp64"]["join_ms_mean"]
                                            / var["fp32_filter"]["join_ms_mean"])
    # the fp32 tier's share of edges left to the fp64 re-test (and to the
    # exact expansion after it)
    _, _, c32 = idx.join_ex(pts, out, counters=True, refine=act.ACT_REFINE_FP32_FILTER)
    var["fp32_filter"]["edges_tested"] = c32["edges"]
    var["fp32_filter"]["fp64_retest_share"] = c32["edge_fp64"] / max(1, c32["edges"])
    var["fp32_filter"]["exact_share"] = c32["edge_exact"] / max(1, c32["edges"])
    # cell-local refinement with pending points resolved by the probe's waves
    wq, tq, _ = time_joins(idx, pts, out, k, 1, pending=act.ACT_PENDING_QUEUE)
    torch.cuda.synchronize()
    var["local_in_probe_queue"] = {"points_per_s": n * k / wq, "join_ms_mean": float(np.mean(tq)),
                                   "identical_to_local": bool(np.array_equal(out.cpu().numpy(),
                                                                             exact_out))}
    log("pair output and per-polygon counts")
    pc, pc_keep = pairs_and_counts_leg(act, [("exact", idx), ("approx4m", idx_a)], pts, k)
    log("the paper's covering configuration, untrained and trained")
    paper_cfg = paper_config_leg(act, P, "c2", pts, out, k)
    log("joins of precomputed cell ids")
    ids_leg = precomputed_ids_leg(act, [("exact", idx), ("approx4m", idx_a)], pts, k, exact_out)
    log("batched join (graph replay)")
    batched = batched_leg(act, idx, pts, exact_out)
    log("serving")
    pools = [synth.workload_points(args.workload, 0, 1 << 22)] * 2
    serving = serving_leg(act, [idx, idx_a], pools, [1e3, 1e4], args.serve_seconds or 2.0)
    serving["indexes"] = "c2 exact, c2 approx@4m"
    

    probe_ms = float(np.mean(prb))
    achieved = BYTES_PER_POINT * n / (probe_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    valu = measured_valu()
    st, sa = idx.stats(), idx_a.stats()
    alu = None
    if valu and "exact" in valu:
        # lane operations per point = wave instructions per 64 points
        ops = valu["exact"] * n / (probe_ms * 1e-3)
        alu = {"bound": "valu", "achieved": ops, "peak": PEAK_VALU_LANE_OPS,
               "unit": "lane-ops/s", "frac": ops / PEAK_VALU_LANE_OPS,
               "valu_instr_per_point": valu["exact"],
               "what": "secondary ceiling: the probe's VALU instructions per point "
                       "(rocprofv3 SQ_INSTS_VALU, committed summary) over its event-timed "
                       "duration, against 1024 SIMDs issuing one wave instruction every 4 "
                       "cycles at 2.4 GHz (fp64 FMA runs at that rate)"}
    res = {
        "metric": "joined points/sec (exact & approx@4m) + HBM roofline %; p50/p99 batch latency",
        "value": value,
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "%s: %d Voronoi polygons over the NYC box (%d edges), %d fp64 "
                               "mixture points resident in HBM, exact join (covering level %d, "
                               "cell-local refinement); approx@4m beside it"
                               % (args.workload, P.n_polys, st["n_edges"], n, EXACT_LEVEL),
                   "n_points": n, "n_polys": P.n_polys, "mode": "exact",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": traffic["exact"] if traffic and "exact" in traffic else None,
                     "kernel": "probe_kernel (exact mode)", "kernel_ms": probe_ms,
                     "bytes_per_point": BYTES_PER_POINT, "points_per_launch": n,
                     "measured_GBps": (traffic["exact"] / (probe_ms * 1e-3) / 1e9
                                       if traffic and "exact" in traffic else None),
                     "join_frac": BYTES_PER_POINT * n / (float(np.mean(tot)) * 1e-3) / 1e9
                                  / PEAK_HBM_GBS,
                     "what": "frac: the probe kernel's algorithmic bytes (20 per point) over "
                             "its event-timed duration, against 8 TB/s (the 40% target is "
                             "stated for the probe); join_frac: the same bytes over the whole "
                             "exact join (probe + resolve); measured_GBps: the kernel's "
                             "rocprofv3-counted HBM bytes over its duration",
                     "alu": alu},
        "latency_ms": {"p50": percentile(tot, 50), "p99": percentile(tot, 99),
                       "what": "one join of all points (one step), HIP events"},
        "batched_exact": batched,
        "serving": serving,
        "exact": {"join_ms_mean": float(np.mean(tot)), "join_ms_median": float(np.median(tot)),
                  "join_ms_min": float(np.min(tot)), "probe_ms_mean": probe_ms,
                  "resolve_ms_mean": float(np.mean(tot) - probe_ms)},
        "approx4m": {"points_per_s": n * args.steps / wall_a,
                     "join_ms_mean": float(np.mean(tot_a)),
                     "join_ms_median": float(np.median(tot_a)),
                     "join_ms_min": float(np.min(tot_a)),
                     "latency_ms": {"p50": percentile(tot_a, 50), "p99": percentile(tot_a, 99)},
                     "roofline_frac": BYTES_PER_POINT * n / (np.mean(prb_a) * 1e-3) / 1e9
                     / PEAK_HBM_GBS,
                     "traffic": traffic["approx"] if traffic and "approx" in traffic else None},
        "refine_variants": var,
        "pairs_and_counts": pc,
        "paper_configuration": paper_cfg,
        "precomputed_ids": ids_leg,
        "counters_exact": ctr,
        "counters_approx4m": ctr_a,
        "index": {"exact": {k2: st[k2] for k2 in ("n_cells", "n_nodes", "node_bytes", "lut_words",
                                                  "local_words", "device_bytes", "max_depth")},
                  "approx4m": {k2: sa[k2] for k2 in ("n_cells", "n_nodes", "node_bytes",
                                                     "lut_words", "device_bytes", "max_depth")},
                  "build_s_exact": t_build_exact, "build_s_approx4m": t_build_approx},
        "copy_calibration": calib,
        "autotuner": tuned,
        "kernel_sources_sha256_16": kernel_source_hash(),
    }
    del pts, out
    torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        ns = min(args.cpu_sample or n, n)
        res["cpu_baseline"], res["parity_vs_oracle"] = cpu_baseline_and_parity(
            P, args.workload, ns, exact_out, pc_keep.get("pairs"), pc_keep.get("counts"))
    if emit:
        print(json.dumps(res), flush=True)
    return res, {"approx4m": idx_a}


def _timed_stream(idx, pts, out, bsz, steps, **kw):
    """Joins of pts in batches of bsz (one step = all batches): wall clock
    over `steps` back-to-back steps, then the HIP-event time of each step of
    a second pass outside that window."""
    import torch
    n = pts.shape[0]

    def once():
        for s in range(0, n, bsz):
            idx.join_ex(pts[s:s + bsz], out[s:s + bsz], **kw)
    once()
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(steps):
        once()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for a, b in ev:
        a.record()
        once()
        b.record()
    torch.cuda.synchronize()
    return wall, [a.elapsed_time(b) for a, b in ev]


def _index_metrics(ctr):
    """The paper's index metrics (Tables III and IV) from join counters:
    false hits, solely true hits, and candidates per point that needs
    refinement."""
    pts = max(1, ctr["points"])
    return {"false_hit_pct": 100.0 * ctr["false_hit"] / pts,
            "solely_true_hit_pct": 100.0 * ctr["solely_true"] / pts,
            "refined_point_pct": 100.0 * ctr["cand_points"] / pts,
            "candidates_per_refined_point": ctr["candidates"] / max(1, ctr["cand_points"])}


def compact_legs(args, keep):
    """Compact forms of the other workloads, in the default run:
    c3: 2^26 points of the 40,000-polygon stream in 2^24 batches, exact
    (covering level 22, with the launch defaults and tuned, and the
    library's default level 20) and approx@1m, with an oracle sample; c4: the first 1,000 batches of the
    uneven-batch mix on the c3 exact index, tuned, one graph replay per
    step, oracle on 1% of the batches plus every batch under 1,000 points;
    c5: the serving sweep at 1e3, 1e4, 1e5 and 4e5 requests/s over the c2
    approx@4m and c3 exact indexes (native load generator)."""
    import numpy as np
    import torch

    import oracle
    import synth
    import paper_1802_09488_amd as act
    legs = {}
    cores = len(os.sched_getaffinity(0))
    log("c3: polygons and indexes")
    P = synth.workload_polygons("c3")
    t0 = time.perf_counter()
    ie = act.build(P, "exact", max_level=EXACT_LEVEL)
    tb_e = time.perf_counter() - t0
    t0 = time.perf_counter()
    it = act.build(P, "exact")  # the library's default covering level, 20
    tb_t = time.perf_counter() - t0
    n, bsz = 1 << 26, 1 << 24
    log("c3: staging %d points" % n)
    pts = _stage_points("c3", n)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    ie.reserve(bsz)
    it.reserve(bsz)
    steps = 5
    c3 = {"n_points": n, "batch": bsz, "steps": steps, "exact_covering_level": EXACT_LEVEL}
    sample = synth.workload_points("c3", 0, 200_000)
    ref = oracle.join(P, sample, nthreads=cores)
    for name, ix, tb in (("exact", ie, tb_e), ("exact_level20", it, tb_t)):
        wall, ms = _timed_stream(ix, pts, out, bsz, steps)
        _, _, ctr = ix.join_ex(pts[:bsz], out[:bsz], counters=True)
        st = ix.stats()
        ok = bool(np.array_equal(out[:200_000].cpu().numpy(), ref.out))
        c3[name] = {"points_per_s": n * steps / wall, "stream_ms": float(np.median(ms)),
                    "roofline_frac": BYTES_PER_POINT * n * steps / wall / 1e9 / PEAK_HBM_GBS,
                    "index_metrics": dict(_index_metrics(ctr), tree_nodes=st["n_nodes"],
                                          image_bytes=st["image_bytes"],
                                          train_splits=st["train_splits"]),
                    "build_s": tb, "oracle_sample_identical": ok}
    wq, _ = _timed_stream(ie, pts, out, bsz, 1, pending=act.ACT_PENDING_QUEUE)
    c3["exact_in_probe_queue_points_per_s"] = n / wq
    # the autotuner's pick for this index on one batch, then the same stream
    tune = ie.tune(pts[:bsz])
    wall, ms = _timed_stream(ie, pts, out, bsz, steps)
    c3["exact_tuned"] = {"points_per_s": n * steps / wall, "stream_ms": float(np.median(ms)),
                         "tuner": tune,
                         "oracle_sample_identical":
                             bool(np.array_equal(out[:200_000].cpu().numpy(), ref.out))}
    t0 = time.perf_counter()
    oracle.join(P, sample, nthreads=cores)
    dt = time.perf_counter() - t0
    c3["cpu_baseline"] = {"value": len(sample) / dt, "unit": "points/s", "cores": cores,
                          "kind": "oracle", "sample": "first 200,000 points of the c3 stream, "
                                                      "exact, %.1f s" % dt}
    del it
    log("c3: approx@1m")
    t0 = time.perf_counter()
    ia = act.build(P, "approx", 1.0)
    tb_a = time.perf_counter() - t0
    wall, ms = _timed_stream(ia, pts, out, bsz, steps)
    oa, pa = ia.join_pairs(pts[:200_000])
    got = set(map(tuple, pa.cpu().numpy().tolist()))
    oa = oa.cpu().numpy()
    got |= {(i, int(o)) for i, o in enumerate(oa) if o >= 0}
    missing = len(set(map(tuple, ref.pair_set().tolist())) - got)
    c3["approx1m"] = {"points_per_s": n * steps / wall, "stream_ms": float(np.median(ms)),
                      "build_s": tb_a, "image_bytes": ia.stats()["image_bytes"],
                      "oracle_pairs_missing_in_sample": missing}
    del ia, pts, out
    torch.cuda.empty_cache()
    legs["c3"] = c3

    log("c4: 1,000 uneven batches")
    sizes = synth.batch_sizes(10_000, 3004)[:1000]
    total = int(sizes.sum())
    pts = _stage_points("c3", total)
    tune = ie.tune(pts[:min(total, 1 << 25)])
    out = torch.full((total,), -9, dtype=torch.int32, device="cuda")
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    batches = [(pts[a:b], out[a:b]) for a, b in zip(bounds[:-1], bounds[1:])]
    desc, tot = act.batch_descriptors(batches)
    ticks = torch.zeros(len(batches) + 1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    ie.batched_reserve(len(batches), tot, stream=s)
    with torch.cuda.stream(s):
        ie.join_batched(desc, tot, ticks=ticks)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ie.join_batched(desc, tot, ticks=ticks)
    hz = act.wall_clock_hz(0)
    ms, p50, p99 = [], [], []
    for _ in range(4):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
        t = ticks.cpu().numpy().view(np.uint64).astype(np.float64)
        lat = (t[1:] - t[0]) / hz * 1e3
        p50.append(float(np.percentile(lat, 50)))
        p99.append(float(np.percentile(lat, 99)))
    rng = np.random.default_rng(3005)
    pick = sorted(set(rng.choice(len(sizes), 10, replace=False).tolist())
                  | set(np.nonzero(sizes < 1000)[0].tolist()))
    sel = np.concatenate([np.arange(bounds[b], bounds[b + 1]) for b in pick])
    sel_t = torch.from_numpy(sel).cuda()
    okc4 = bool(np.array_equal(out[sel_t].cpu().numpy(),
                               oracle.join(P, pts[sel_t].cpu().numpy(), nthreads=cores).out))
    med = float(np.median(ms[1:]))
    legs["c4"] = {"batches": len(sizes), "n_points": total, "graph_replay_ms": med,
                  "points_per_s": total / (med * 1e-3),
                  "batch_latency_ms": {"p50": float(np.median(p50)), "p99": float(np.median(p99)),
                                       "what": "per-batch completion tick minus the join's "
                                               "start tick"},
                  "tuner": tune, "oracle": {"batches_checked": len(pick),
                                            "points_checked": int(len(sel)), "identical": okc4}}
    del g, pts, out, batches, desc
    torch.cuda.empty_cache()

    log("c5: serving sweep")
    pools = [synth.workload_points("c2", 0, 1 << 22), synth.workload_points("c3", 0, 1 << 22)]
    srv = serving_leg(act, [keep["approx4m"], ie], pools, [1e3, 1e4, 1e5, 4e5], 2.0)
    srv["indexes"] = "c2 approx@4m, c3 exact"
    legs["c5"] = srv
    return legs


def _stage_points(workload, n, step=1 << 24):
    """Points [0, n) of a workload's stream, generated on the host and
    staged in HBM."""
    import torch

    import synth
    pts = torch.empty((n, 2), dtype=torch.float64, device="cuda")
    for s in range(0, n, step):
        e = min(n, s + step)
        pts[s:e].copy_(torch.from_numpy(synth.workload_points(workload, s, e)))
    torch.cuda.synchronize()
    return pts


def _line(metric_value, steps, warmup, ms_per_step, config, **extra):
    res = {"metric": "joined points/sec (exact & approx@4m) + HBM roofline %; "
                     "p50/p99 batch latency",
           "value": metric_value, "unit": "points/s", "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
           "config": config}
    res.update(extra)
    print(json.dumps(res), flush=True)


def run_c3(args):
    """40,000 polygons; 1e9 points staged in HBM (16 GB) and joined as 60
    batches of 2^24 (one step = the whole stream): exact (cell-local, and
    the fp32-filter and all-fp64 refinements over all edges) and approx@1m."""
    import numpy as np
    import torch

    import oracle
    import synth
    import paper_1802_09488_amd as act
    w = synth.WORKLOADS["c3"]
    n = args.points or w["n_points"]
    bsz = w["batch"]
    P = synth.workload_polygons("c3")
    t0 = time.perf_counter()
    idx = act.build(P, "exact", max_level=EXACT_LEVEL)
    tb_e = time.perf_counter() - t0
    t0 = time.perf_counter()
    idx_a = act.build(P, "approx", 1.0)
    tb_a = time.perf_counter() - t0
    log("staging %d points" % n)
    pts = _stage_points("c3", n)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    idx.reserve(bsz)

    def stream(ix, **kw):
        for s in range(0, n, bsz):
            ix.join_ex(pts[s:s + bsz], out[s:s + bsz], **kw)

    def timed(ix, steps, **kw):
        stream(ix, **kw)
        torch.cuda.synchronize()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        t = time.perf_counter()
        for a, b in ev:
            a.record()
            stream(ix, **kw)
            b.record()
        torch.cuda.synchronize()
        return time.perf_counter() - t, [a.elapsed_time(b) for a, b in ev]

    steps = max(1, min(args.steps, 3))
    wall, ms = timed(idx, steps)
    sample = synth.workload_points("c3", 0, 200_000)
    ref = oracle.join(P, sample)
    torch.cuda.synchronize()
    ok = bool(np.array_equal(out[:200_000].cpu().numpy(), ref.out))
    var = {}
    for name, mode in (("fp32_filter", act.ACT_REFINE_FP32_FILTER), ("fp64", act.ACT_REFINE_FP64)):
        wv, mv = timed(idx, 1, refine=mode)
        var[name] = {"points_per_s": n / wv, "stream_ms": float(np.mean(mv))}
    var["fp32_filter_over_fp64_speedup"] = var["fp64"]["stream_ms"] / var["fp32_filter"]["stream_ms"]
    wq, mq = timed(idx, 1, pending=act.ACT_PENDING_QUEUE)
    var["local_in_probe_queue"] = {"points_per_s": n / wq, "stream_ms": float(np.mean(mq))}
    wa, ma = timed(idx_a, steps)
    cores = len(os.sched_getaffinity(0))
    t0 = time.perf_counter()
    oracle.join(P, sample, nthreads=cores)
    dt = time.perf_counter() - t0
    st, sa = idx.stats(), idx_a.stats()
    _line(n * steps / wall, steps, 1, 1000 * wall / steps,
          {"workload": "c3: 40,000 Voronoi polygons over the NYC box, %d fp64 mixture points "
                       "staged in HBM, joined in batches of 2^24, exact (cell-local refinement)"
                       % n, "n_points": n, "batch": bsz, "n_polys": P.n_polys,
           "parallelism": "single GPU"},
          approx1m={"points_per_s": n * steps / wa, "stream_ms": float(np.mean(ma))},
          refine_variants=var, parity_vs_oracle={"points_checked": 200_000, "ok": ok},
          index={"exact": {k: st[k] for k in ("n_cells", "n_nodes", "node_bytes",
                                                "device_bytes")},
                 "approx1m": {k: sa[k] for k in ("n_cells", "n_nodes", "node_bytes",
                                                   "device_bytes")},
                 "build_s_exact": tb_e, "build_s_approx1m": tb_a},
          cpu_baseline={"value": len(sample) / dt, "unit": "points/s", "cores": cores,
                        "kind": "oracle",
                        "sample": "first 200,000 points of the c3 stream, exact, %.1f s" % dt})


def run_c4(args):
    """10,000 batches of floor(exp(U(0, ln 1e6))) points (seed 3004) of the
    c3 stream against the 40,000-polygon exact index: the autotuner picks the
    launch shape on a sample, then one batched join is captured in a HIP
    graph and replayed (one step = one replay)."""
    import numpy as np
    import torch

    import synth
    import paper_1802_09488_amd as act
    P = synth.workload_polygons("c3")
    idx = act.build(P, "exact", max_level=EXACT_LEVEL)
    sizes = synth.batch_sizes(10_000, 3004)
    total = int(sizes.sum())
    log("staging %d points in %d batches" % (total, len(sizes)))
    pts = _stage_points("c3", total)
    # a sample large enough that launch shapes separate beyond timing noise
    tune = idx.tune(pts[:1 << 25])
    out = torch.empty(total, dtype=torch.int32, device="cuda")
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    batches = [(pts[a:b], out[a:b]) for a, b in zip(bounds[:-1], bounds[1:])]
    desc, tot = act.batch_descriptors(batches)
    ticks = torch.zeros(len(batches) + 1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    idx.batched_reserve(len(batches), tot, stream=s)
    with torch.cuda.stream(s):
        idx.join_batched(desc, tot, ticks=ticks)
    s.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        idx.join_batched(desc, tot, ticks=ticks)
    hz = act.wall_clock_hz(0)
    steps = max(1, args.steps)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    ms, p50, p99 = [], [], []
    t_all = time.perf_counter()
    for _ in range(steps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        torch.cuda.synchronize()
        ms.append(a.elapsed_time(b))
        t = ticks.cpu().numpy().view(np.uint64).astype(np.float64)
        lat = (t[1:] - t[0]) / hz * 1e3
        p50.append(float(np.percentile(lat, 50)))
        p99.append(float(np.percentile(lat, 99)))
    wall = time.perf_counter() - t_all
    single = idx.join(pts[:2_000_000])
    same = bool(torch.equal(single, out[:2_000_000]))
    _line(total / (float(np.median(ms)) * 1e-3), steps, args.warmup, float(np.median(ms)),
          {"workload": "c4: 10,000 uneven batches (%d points) of the c3 stream, 40,000-polygon "
                       "exact index, one batched join per step (HIP graph replay)" % total,
           "batches": len(sizes), "n_points": total, "parallelism": "single GPU"},
          batch_latency_ms={"p50": float(np.median(p50)), "p99": float(np.median(p99)),
                            "what": "per-batch completion tick minus the join's start tick"},
          wall_s=wall, tuner=tune, identical_to_single_join=same)


def run_c5(args):
    """Serving: Poisson arrivals at 1e3 ... 1.6e6 requests/s of
    floor(exp(U(0, ln 65536))) points, each aimed at the 290-polygon
    approx@4m index or the 40,000-polygon exact index, replayed by the
    native load generator for 4 s per rate."""
    import synth
    import paper_1802_09488_amd as act
    ia = act.build(synth.workload_polygons("c2"), "approx", 4.0)
    ie = act.build(synth.workload_polygons("c3"), "exact", max_level=EXACT_LEVEL)
    pools = [synth.workload_points("c2", 0, 1 << 22), synth.workload_points("c3", 0, 1 << 22)]
    sec = args.serve_seconds or 4.0
    srv = serving_leg(act, [ia, ie], pools, [1e3, 1e4, 5e4, 1e5, 2e5, 4e5, 8e5, 1.6e6], sec)
    srv["indexes"] = "c2 approx@4m, c3 exact"
    best = max(r["points_per_s"] for r in srv["runs"])
    _line(best, len(srv["runs"]), 0, 1000.0 * sec,
          {"workload": "c5: serving, Poisson requests of 1..65,536 points over two resident "
                       "indexes (c2 approx@4m, c3 exact)", "parallelism": "single GPU"},
          serving=srv)


# ------------------------------------------------------------ profile summaries

def _csv_rows(d, suffix):
    files = glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True)
    if not files:
        raise SystemExit("no *%s under %s" % (suffix, d))
    rows = []
    for f in files:
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _short(name):
    name = re.sub(r"\(.*", "", name)
    return name.replace("void ", "").replace("act::", "")


def summarize_trace(d):
    """Per (kernel, launch grid): calls and durations, from the kernel trace."""
    import numpy as np
    rows = _csv_rows(d, "kernel_trace.csv")
    groups = {}
    for r in rows:
        key = (_short(r["Kernel_Name"]), int(r["Grid_Size_X"]), int(r["Workgroup_Size_X"]))
        groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    print("| kernel | grid (threads) | block | calls | avg (us) | min (us) | max (us) | total (ms) |")
    print("|---|---|---|---|---|---|---|---|")
    for (name, grid, blk), v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:14]:
        v = np.asarray(v)
        print("| %s | %d | %d | %d | %.1f | %.1f | %.1f | %.2f |" % (
            name, grid, blk, len(v), v.mean(), v.min(), v.max(), v.sum() / 1e3))


def _act_kernel_args(name):
    m = re.search(r"(probe_kernel|resolve_kernel|resolve_list_kernel)<([^>]*)>", name)
    if not m:
        return None, None
    return m.group(1), [x.strip() for x in m.group(2).split(",")]


def _lean_act_kernel(name):
    """This library's kernels without counters and pair output (the FULL
    template argument: third of probe_kernel, second of resolve_kernel,
    first of resolve_list_kernel; 0 = lean)."""
    kind, a = _act_kernel_args(name)
    if kind is None:
        return False
    full = {"probe_kernel": 2, "resolve_kernel": 1, "resolve_list_kernel": 0}[kind]
    return a[full] in ("0", "false")


def _kernel_label(name):
    """Short label of a lean, unbatched kernel of this library (None for the
    others): probe_kernel<mode, LDS levels, full, points per lane, batched,
    ids> with mode 0 approximate, 1 exact with the pending mask, 2 exact with
    the probe's queues, 3 exact with per-wave pending lists (the default),
    4 and 5 the count joins; resolve_kernel<local, full, batched>;
    resolve_list_kernel<full, count>."""
    kind, a = _act_kernel_args(name)
    if kind is None or not _lean_act_kernel(name):
        return None
    if kind == "probe_kernel":
        if a[4] != "false":
            return None
        label = "probe_kernel " + {"0": "approx", "1": "exact-mask", "2": "exact-queue",
                                   "3": "exact", "4": "count approx", "5": "count exact"}[a[0]]
        return label + (" ids" if len(a) > 5 and a[5] == "true" else "")
    if kind == "resolve_kernel":
        if a[2] != "false":
            return None
        return "resolve_kernel %s" % ("local" if a[0] == "true" else "all-edges")
    return "resolve_list_kernel" + (" count" if len(a) > 1 and a[1] == "true" else "")


def summarize_counters(dirs, points_per_launch):
    """Issue and L2 counters of the largest launches of each lean kernel
    (medians over those launches; counting kernels and small grids left
    out): VALU and SALU instructions (per 64 points when the points per
    launch are given), VALU busy = SQ_INSTS_VALU x 4 cycles / (1024 SIMDs x
    GRBM_GUI_ACTIVE / 8), the share of wave time waiting on instruction
    issue (SQ_WAIT_INST_ANY / SQ_WAVE_CYCLES) and the L2 hit rate
    (TCC_HIT_sum / TCC_REQ_sum)."""
    import numpy as np
    vals, grids = {}, {}
    for d in dirs:
        for r in _csv_rows(d, "counter_collection.csv"):
            k, g = _short(r["Kernel_Name"]), int(r["Grid_Size"])
            if not _lean_act_kernel(k):
                continue  # torch's and the runtime's kernels, the counting kernels
            if g > grids.get(k, -1):
                grids[k], vals[k] = g, {}
            if g == grids[k]:
                vals[k].setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    print("kernel sources sha256/16: `%s`" % kernel_source_hash())
    print()
    unit = "per 64 points" if points_per_launch else "per launch"
    print("| kernel | grid | VALU instr. %s | SALU instr. %s | VALU busy | issue wait | "
          "L2 hit rate |" % (unit, unit))
    print("|---|---|---|---|---|---|---|")
    for k in sorted(vals):
        m = {c: float(np.median(v)) for c, v in vals[k].items()}
        div = points_per_launch / 64.0 if points_per_launch else 1.0
        cyc = m.get("GRBM_GUI_ACTIVE", 0.0) / 8.0

        def f(x, fmt):
            return fmt % x if x is not None else "-"
        print("| %s | %d | %s | %s | %s | %s | %s |" % (
            k, grids[k],
            f(m["SQ_INSTS_VALU"] / div if "SQ_INSTS_VALU" in m else None, "%.4g"),
            f(m["SQ_INSTS_SALU"] / div if "SQ_INSTS_SALU" in m else None, "%.4g"),
            f(100 * m["SQ_INSTS_VALU"] * 4 / (1024 * cyc) if cyc and "SQ_INSTS_VALU" in m
              else None, "%.0f%%"),
            f(100 * m["SQ_WAIT_INST_ANY"] / m["SQ_WAVE_CYCLES"]
              if "SQ_WAIT_INST_ANY" in m and m.get("SQ_WAVE_CYCLES") else None, "%.0f%%"),
            f(100 * m["TCC_HIT_sum"] / m["TCC_REQ_sum"]
              if "TCC_HIT_sum" in m and m.get("TCC_REQ_sum") else None, "%.0f%%")))


def summarize_pmc(fdir, wdir):
    """HBM bytes per launch of the probe kernels: FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch), each scaled by the factor that makes the same
    counter read COPY_BYTES for the calibration copy."""
    import numpy as np
    per = {}
    for d, ctr in ((fdir, "FETCH_SIZE"), (wdir, "WRITE_SIZE")):
        vals, grids = {}, {}
        for r in _csv_rows(d, "counter_collection.csv"):
            if r["Counter_Name"] != ctr:
                continue
            k, g = r["Kernel_Name"], int(r["Grid_Size"])
            if g > grids.get(k, -1):  # keep the full-size launches of each kernel
                grids[k], vals[k] = g, []
            if g == grids[k]:
                vals[k].append(float(r["Counter_Value"]) * 1024.0)
        copies = max((v for k, v in vals.items() if "copyBuffer" in k), key=max)
        cal = COPY_BYTES / max(copies)
        per[ctr] = (cal, vals)
    fcal, fv = per["FETCH_SIZE"]
    wcal, wv = per["WRITE_SIZE"]
    print("kernel sources sha256/16: `%s`" % kernel_source_hash())
    print()
    print("calibration (1 GiB device-to-device copy): FETCH_SIZE x %.4f, WRITE_SIZE x %.4f"
          % (fcal, wcal))
    print()
    print("| kernel | HBM bytes per launch | fetch (scaled) | write (scaled) | launches |")
    print("|---|---|---|---|---|")
    for k in sorted(fv):
        label = _kernel_label(k)
        if label is None:
            continue  # other kernels, and the counting variants
        f = float(np.median(fv[k])) * fcal
        wr = float(np.median(wv.get(k, [0.0]))) * wcal
        print("| %s | %.4g | %.4g | %.4g | %d |" % (label, f + wr, f, wr, len(fv[k])))

if __name__ == "__main__":
    main()
