"""GPU parity: the HIP probe (through the C ABI) vs the brute-force oracle.

Exact mode must match bit for bit: out[i] (lowest covering id or -1) and the
set of further (point, polygon) pairs. Approximate mode must respect its
guarantee: no covering polygon missed, and every extra pair's point lies
within precision_m of that polygon's boundary.
"""
import os

import numpy as np
import pytest

import oracle
import synth
from oracle import cellid as C

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def act():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_09488_amd as act
    return act


_IDX = {}


def act_mod():
    import paper_1802_09488_amd
    return paper_1802_09488_amd


def index(act, w, mode, prec=0.0):
    key = (w, mode, prec)
    if key not in _IDX:
        _IDX[key] = (synth.workload_polygons(w), None)
        P = _IDX[key][0]
        _IDX[key] = (P, act.build(P, mode, prec))
    return _IDX[key]


def gpu_join(idx, pts, **kw):
    t = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    try:
        out, pairs, ctr = idx.join_ex(t, capacity=max(4096, len(pts) // 4), **kw)
    except act_mod().ActError as e:
        if e.code != -5:
            raise
        out, pairs, ctr = idx.join_ex(t, capacity=e.needed, **kw)
    torch.cuda.synchronize()
    pr = pairs.cpu().numpy() if pairs is not None else np.zeros((0, 2), np.int64)
    order = np.lexsort((pr[:, 1], pr[:, 0])) if len(pr) else np.zeros(0, np.int64)
    return out.cpu().numpy(), pr[order], ctr


def assert_exact(P, pts, out, pairs, label=""):
    ref = oracle.join(P, pts)
    bad = np.nonzero(out != ref.out)[0]
    assert bad.size == 0, "%s: %d mismatches, first %s: gpu %s oracle %s" % (
        label, bad.size, bad[:5], out[bad[:5]], ref.out[bad[:5]])
    assert np.array_equal(pairs, ref.pairs), "%s: pair sets differ (%d vs %d)" % (
        label, len(pairs), len(ref.pairs))
    return ref


def assert_approx(P, pts, out, pairs, prec, label=""):
    ref = oracle.join(P, pts)
    got = set(map(tuple, pairs.tolist()))
    got |= {(i, int(o)) for i, o in enumerate(out) if o >= 0}
    want = set(map(tuple, ref.pair_set().tolist()))
    missing = want - got
    assert not missing, "%s: %d covering pairs missing, e.g. %s" % (label, len(missing),
                                                                     sorted(missing)[:3])
    extra = np.asarray(sorted(got - want), dtype=np.int64).reshape(-1, 2)
    if len(extra):
        d = oracle.boundary_dist_pairs(P, pts, extra)
        assert d.max() <= prec + 1e-6, "%s: extra pair %.3f m from boundary" % (label, d.max())
    # out[i] is the lowest reported id
    lowest = {}
    for i, p in got:
        lowest[i] = min(lowest.get(i, 1 << 40), p)
    for i, o in enumerate(out):
        assert o == lowest.get(i, -1)
    return len(extra), len(got)


def edge_case_points(P, rng):
    """Vertices (on boundaries, shared by neighbours; hole vertices where the
    workload has holes), vertices moved by one ulp in either coordinate,
    edge midpoints (within rounding of an edge), invalid and out-of-domain
    points, points outside the box."""
    v = P.verts
    mids = 0.5 * (v[:-1] + v[1:])  # near (not exactly on) edges
    k = rng.choice(len(v), min(len(v), 4000), replace=False)
    nudged = v[k] + rng.integers(-1, 2, (len(k), 2)) * np.spacing(v[k])
    bad = np.array([[np.nan, -74.0], [40.7, np.inf], [-np.inf, 0], [91.0, -74.0],
                    [40.7, -181.0], [90.0, 180.0], [-90.0, -180.0], [0.0, 0.0],
                    [40.7, 106.0], [-40.7, -74.0]])
    outside = np.stack([rng.uniform(39, 42, 500), rng.uniform(-75.5, -72.5, 500)], 1)
    return np.concatenate([v, nudged, mids, bad, outside])


def test_c1_exact_all_points(act):
    P, idx = index(act, "c1", "exact")
    pts = synth.workload_points("c1")
    out, pairs, ctr = gpu_join(idx, pts, counters=True)
    assert_exact(P, pts, out, pairs, "c1")
    assert ctr["points"] == len(pts)


def test_c1_exact_edge_cases(act):
    P, idx = index(act, "c1", "exact")
    pts = edge_case_points(P, np.random.default_rng(3))
    out, pairs, _ = gpu_join(idx, pts)
    ref = assert_exact(P, pts, out, pairs, "c1-edges")
    assert len(ref.pairs) > 100  # shared vertices really produce multi-matches


REFINE_MODES = ["ACT_REFINE_LOCAL", "ACT_REFINE_FP32_FILTER", "ACT_REFINE_FP64"]


@pytest.mark.parametrize("mode,pending", [("ACT_REFINE_LOCAL", "ACT_PENDING_QUEUE"),
                                          ("ACT_REFINE_LOCAL", "ACT_PENDING_KERNEL"),
                                          ("ACT_REFINE_FP32_FILTER", "ACT_PENDING_AUTO"),
                                          ("ACT_REFINE_FP64", "ACT_PENDING_AUTO")])
def test_c1_refine_modes_exact(act, mode, pending):
    """Every refinement mode gives the oracle's result, edge cases included
    (cell-local refinement inside the probe and in a second kernel)."""
    P, idx = index(act, "c1", "exact")
    pts = np.concatenate([synth.workload_points("c1"), edge_case_points(P, np.random.default_rng(4))])
    out, pairs, _ = gpu_join(idx, pts, refine=getattr(act, mode), pending=getattr(act, pending))
    assert_exact(P, pts, out, pairs, "c1-" + mode)


@pytest.mark.parametrize("mode", REFINE_MODES)
def test_c2_refine_modes_exact(act, mode):
    P, idx = index(act, "c2", "exact")
    pts = np.concatenate([synth.workload_points("c2", 0, 200000),
                          edge_case_points(P, np.random.default_rng(5))])
    out, pairs, _ = gpu_join(idx, pts, refine=getattr(act, mode))
    assert_exact(P, pts, out, pairs, "c2-" + mode)


@pytest.mark.parametrize("n", [1, 2, 63, 64, 65, 255, 257, 4097, 100003])
def test_ragged_sizes(act, n):
    P, idx = index(act, "c1", "exact")
    pts = synth.uniform_points(0, n, seed=91)
    out, pairs, _ = gpu_join(idx, pts)
    assert_exact(P, pts, out, pairs, "n=%d" % n)


def test_empty_batch(act):
    P, idx = index(act, "c1", "exact")
    t = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
    out = idx.join(t)
    torch.cuda.synchronize()
    assert out.shape == (0,)


@pytest.mark.parametrize("mode,prec", [("exact", 0.0), ("approx", 4.0)])
def test_launch_shapes_and_repeats_identical(act, mode, prec):
    """Output does not depend on the grid size, the LDS-staged trie depth or
    the run (determinism / race check)."""
    P, idx = index(act, "c2", mode, prec)
    pts = synth.workload_points("c2", 0, 300000)
    base = gpu_join(idx, pts)
    fits = []
    for lds in (0, 1, 2):
        try:
            gpu_join(idx, pts[:64], lds_levels=lds)
            fits.append(lds)
        except act.ActError as e:  # top levels larger than the LDS budget
            assert e.code == -7
    assert 0 in fits and 1 in fits
    for grid in (1, 7, 256, 0):
        for lds in fits:
            for npl in (1, 2):
                for _ in range(2):
                    o = gpu_join(idx, pts, grid=grid, lds_levels=lds, points_per_lane=npl)
                    assert np.array_equal(o[0], base[0]) and np.array_equal(o[1], base[1]), \
                        (grid, lds, npl)


def test_c1_approx_guarantee(act):
    P, idx = index(act, "c1", "approx", 4.0)
    pts = np.concatenate([synth.workload_points("c1"), edge_case_points(P, np.random.default_rng(5))])
    out, pairs, _ = gpu_join(idx, pts)
    assert_approx(P, pts, out, pairs, 4.0, "c1-approx4")


def test_c2_exact_sample(act):
    P, idx = index(act, "c2", "exact")
    pts = np.concatenate([synth.workload_points("c2", 0, 1_000_000),
                          edge_case_points(P, np.random.default_rng(6))])
    out, pairs, ctr = gpu_join(idx, pts, counters=True)
    assert_exact(P, pts, out, pairs, "c2")
    assert ctr["candidates"] > 0 and ctr["cand_points"] > 0
    # over all edges with the fp32 filter: some edges, not all, go to fp64
    out2, pairs2, ctr2 = gpu_join(idx, pts, counters=True, refine=act.ACT_REFINE_FP32_FILTER)
    assert np.array_equal(out2, out) and np.array_equal(pairs2, pairs)
    assert 0 < ctr2["edge_fp64"] < ctr2["edges"], ctr2
    assert ctr2["edge_exact"] <= ctr2["edge_fp64"]


def test_c2_approx_sample(act):
    P, idx = index(act, "c2", "approx", 4.0)
    pts = synth.workload_points("c2", 0, 1_000_000)
    out, pairs, _ = gpu_join(idx, pts)
    n_extra, n_pairs = assert_approx(P, pts, out, pairs, 4.0, "c2-approx4")
    assert n_extra < 0.05 * n_pairs


def test_c2_full_size_sampled(act):
    """All 1e8 points of the workload in one launch (the benchmark's
    configuration); the oracle checks 200k seeded random positions, and the
    cell-local, fp32-filter and all-fp64 refinements agree everywhere."""
    P, idx = index(act, "c2", "exact")
    n = synth.WORKLOADS["c2"]["n_points"]
    pts = torch.from_numpy(synth.workload_points("c2", 0, n)).cuda()
    out = idx.join(pts)
    for mode in (act.ACT_REFINE_FP32_FILTER, act.ACT_REFINE_FP64):
        other, _, _ = idx.join_ex(pts, refine=mode)
        torch.cuda.synchronize()
        assert torch.equal(out, other), mode
        del other
    rng = np.random.default_rng(7)
    sel = np.sort(rng.choice(n, 200000, replace=False))
    sp = pts[torch.from_numpy(sel).cuda()].cpu().numpy()
    ref = oracle.join(P, sp)
    assert np.array_equal(out[torch.from_numpy(sel).cuda()].cpu().numpy(), ref.out)
    del pts


def test_cell_ids_match_reference(act):
    rng = np.random.default_rng(8)
    pts = np.concatenate([
        np.stack([rng.uniform(-90, 90, 300000), rng.uniform(-180, 180, 300000)], 1),
        synth.workload_points("c2", 0, 300000),
        np.array([[0, 0], [90, 0], [-90, 0], [0, 180], [0, -180], [0, 45], [35.26438968, 45.0]]),
    ])
    t = torch.from_numpy(pts).cuda()
    got = act.cell_ids(t).cpu().numpy().view(np.uint64)
    want = C.cell_ids(pts[:, 0], pts[:, 1])
    diff = np.nonzero(got != want)[0]
    # ids may differ only where the point sits within rounding of a leaf
    # boundary (different sin/cos implementations); the GPU's leaf must then
    # be a neighbour of the reference leaf
    assert diff.size < 1e-4 * len(pts), diff.size
    if diff.size:
        f1, i1, j1 = C.decode_leaf(got[diff])
        f2, i2, j2 = C.decode_leaf(want[diff])
        same = f1 == f2
        assert np.all(np.abs(i1 - i2)[same] <= 1) and np.all(np.abs(j1 - j2)[same] <= 1)
    bad = torch.tensor([[np.nan, 0.0], [0.0, 200.0]], dtype=torch.float64, device="cuda")
    assert act.cell_ids(bad).cpu().tolist() == [0, 0]


def overlapping_polygons(seed=12, n=9):
    """n star-shaped polygons around nearly the same centre, with holes in
    some: cells near their crowded boundaries reference many polygons, many
    of them as candidates (lookup-table lists longer than three)."""
    rng = np.random.default_rng(seed)
    polys = []
    for k in range(n):
        c = np.array([40.70, -73.95]) + rng.normal(0, 0.002, 2)
        m = int(rng.integers(8, 40))
        ang = np.sort(rng.uniform(0, 2 * np.pi, m))
        rad = 0.01 * rng.uniform(0.7, 1.3, m)
        outer = np.stack([c[0] + rad * np.sin(ang), c[1] + rad * np.cos(ang) / 0.76], 1)
        rings = [outer]
        if k % 3 == 0:
            hang = np.sort(rng.uniform(0, 2 * np.pi, 12))
            hrad = 0.002 * rng.uniform(0.8, 1.2, 12)
            rings.append(np.stack([c[0] + hrad * np.sin(hang), c[1] + hrad * np.cos(hang) / 0.76], 1))
        polys.append(rings)
    return synth.Polygons.from_rings(polys)


@pytest.mark.parametrize("pass_points,mode,queue", [(0, "ACT_REFINE_LOCAL", True),
                                                    (1000, "ACT_REFINE_LOCAL", False),
                                                    (4097, "ACT_REFINE_FP32_FILTER", False),
                                                    (0, "ACT_REFINE_FP64", False)])
def test_overlapping_polygons_long_candidate_lists(act, pass_points, mode, queue):
    """Exact parity where cells hold up to n references (long lookup-table
    lists, several matches per point, most points pending), resolved inside
    the probe, and by a second kernel in one pass and in many short passes
    (pair output then carries the pass offset)."""
    P = overlapping_polygons()
    idx = act.build(P, "exact", max_level=16)
    st = idx.stats()
    assert st["max_refs"] >= 5
    rng = np.random.default_rng(13)
    pts = np.concatenate([
        np.stack([rng.uniform(40.68, 40.72, 200000), rng.uniform(-73.98, -73.92, 200000)], 1),
        P.verts])
    kw = dict(pass_points=pass_points, refine=getattr(act, mode),
              pending=act.ACT_PENDING_QUEUE if queue else act.ACT_PENDING_KERNEL)
    out, pairs, ctr = gpu_join(idx, pts, counters=True, **kw)
    ref = assert_exact(P, pts, out, pairs, "overlap pass=%d %s" % (pass_points, mode))
    assert ref.cnt.max() >= 5
    assert ctr["points"] == len(pts) and ctr["cand_points"] > 0
    # a repeated join on the same stream reuses the workspace
    out2, pairs2, _ = gpu_join(idx, pts, **kw)
    assert np.array_equal(out2, out)
    assert np.array_equal(np.unique(pairs2, axis=0), np.unique(pairs, axis=0))


@pytest.mark.parametrize("mode", ["exact", "approx"])
def test_small_and_ragged_lengths(act, mode):
    """Joins whose length leaves waves with no tile, one tile, or a ragged
    last tile (lanes without a point), at both lane widths and at grids that
    give every wave many tiles or none, through the lean kernels (plain
    joins) and the full ones (pairs): every out equals the same points'
    share of the reference (the oracle in exact mode, the full kernel's
    large join, checked against the oracle elsewhere, in approximate mode)."""
    P, idx = index(act, "c2", mode, 0.0 if mode == "exact" else 4.0)
    pts = np.concatenate([synth.workload_points("c2", 0, 70_000),
                          edge_case_points(P, np.random.default_rng(18))[:5000]])
    full, full_pairs, _ = gpu_join(idx, pts)
    if mode == "exact":
        assert np.array_equal(full, oracle.join(P, pts).out)
    t = torch.from_numpy(pts).cuda()
    for n in (1, 2, 63, 64, 65, 127, 128, 129, 255, 256, 257, 1000, 4097, 70_001):
        for npl in (1, 2):
            for grid in (1, 3, 0, 4096):
                # outputs are written through buffers sized to each tile:
                # nothing past n may change
                buf = torch.full((n + 200,), -7, dtype=torch.int32, device="cuda")
                lean, _, _ = idx.join_ex(t[:n], out=buf[:n], points_per_lane=npl, grid=grid)
                torch.cuda.synchronize()
                assert np.array_equal(lean.cpu().numpy(), full[:n]), (n, npl, grid)
                assert bool((buf[n:] == -7).all()), (n, npl, grid)
            o, pr, _ = gpu_join(idx, pts[:n], points_per_lane=npl)
            assert np.array_equal(o, full[:n]), (n, npl)
            assert np.array_equal(pr, full_pairs[full_pairs[:, 0] < n]), (n, npl)


def test_workspace_reserve_and_passes(act):
    """With pending points resolved by the second kernel, a reserved
    workspace smaller than the batch splits the join into passes; results
    equal the one-pass join and the join that resolves in the probe."""
    P, idx = index(act, "c2", "exact")
    pts = torch.from_numpy(synth.workload_points("c2", 0, 1_000_003)).cuda()
    one = idx.join(pts)
    queued, _, _ = idx.join_ex(pts, pending=act.ACT_PENDING_QUEUE)
    idx2 = act.build(P, "exact")
    idx2.reserve(100_000)
    many, _, _ = idx2.join_ex(pts, pending=act.ACT_PENDING_KERNEL)
    torch.cuda.synchronize()
    assert torch.equal(one, many) and torch.equal(one, queued)


def test_pending_queue_and_kernel_agree(act):
    """Pending points resolved inside the probe and by the resolve kernel:
    identical outputs, pairs and counters, at both lane widths."""
    P, idx = index(act, "c2", "exact")
    pts = np.concatenate([synth.workload_points("c2", 0, 1_000_000),
                          edge_case_points(P, np.random.default_rng(16))])
    for npl in (1, 2):
        o1, p1, c1 = gpu_join(idx, pts, counters=True, points_per_lane=npl,
                              pending=act.ACT_PENDING_QUEUE)
        o2, p2, c2 = gpu_join(idx, pts, counters=True, points_per_lane=npl,
                              pending=act.ACT_PENDING_KERNEL)
        assert np.array_equal(o1, o2) and np.array_equal(p1, p2)
        assert c1 == c2, (c1, c2)
        t = torch.from_numpy(pts).cuda()
        for pend in (act.ACT_PENDING_QUEUE, act.ACT_PENDING_KERNEL):  # lean kernels
            lean, _, _ = idx.join_ex(t, points_per_lane=npl, pending=pend)
            torch.cuda.synchronize()
            assert np.array_equal(lean.cpu().numpy(), o1), (npl, pend)
        assert c1["cand_points"] > 1000


def test_pending_lists_and_mask_agree(act):
    """Exact joins record pending points in per-wave lists unless the probe
    grid has more waves than the lists hold (grid > 4096): then in the
    pending mask. Both routes give identical outputs, pairs and counters,
    lean and counting, and a sample of points matches the oracle."""
    P, idx = index(act, "c2", "exact")
    pts = np.concatenate([synth.workload_points("c2", 0, 10_700_000),
                          edge_case_points(P, np.random.default_rng(17))])
    t = torch.from_numpy(pts).cuda()
    for npl in (1, 2):
        # grid 5200 has 83,200 waves (mask); with two points per lane it
        # still gets 5200 blocks of tiles (10.7e6 / 2048 > 5200)
        o1, p1, c1 = gpu_join(idx, pts, counters=True, points_per_lane=npl, grid=1024,
                              pending=act.ACT_PENDING_KERNEL)
        o2, p2, c2 = gpu_join(idx, pts, counters=True, points_per_lane=npl, grid=5200,
                              pending=act.ACT_PENDING_KERNEL)
        assert np.array_equal(o1, o2) and np.array_equal(p1, p2), npl
        assert c1 == c2, (c1, c2)
        for g in (1024, 5200):  # lean kernels
            lean, _, _ = idx.join_ex(t, points_per_lane=npl, grid=g,
                                     pending=act.ACT_PENDING_KERNEL)
            torch.cuda.synchronize()
            assert np.array_equal(lean.cpu().numpy(), o1), (npl, g)
        assert c1["cand_points"] > 10000
    rng = np.random.default_rng(18)
    sample = np.concatenate([rng.choice(len(pts), 20000, replace=False),
                             np.arange(len(pts) - 300, len(pts))])
    ref = oracle.join(P, pts[sample])
    assert np.array_equal(o1[sample], ref.out)


def test_concurrent_streams_share_an_index(act):
    """Joins of one exact index enqueued on two streams at once (each stream
    has its own pending workspace), with the pending points listed and
    resolved by a second kernel on one and resolved in the probe on the
    other: every result equals the one-stream join's."""
    P, idx = index(act, "c2", "exact")
    a = torch.from_numpy(synth.workload_points("c2", 0, 2_000_000)).cuda()
    b = torch.from_numpy(synth.workload_points("c2", 2_000_000, 3_500_000)).cuda()
    ref_a, ref_b = idx.join(a).cpu().numpy(), idx.join(b).cpu().numpy()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    for _ in range(3):
        with torch.cuda.stream(s1):
            oa, _, _ = idx.join_ex(a, pending=act.ACT_PENDING_KERNEL, stream=s1)
        with torch.cuda.stream(s2):
            ob, _, _ = idx.join_ex(b, pending=act.ACT_PENDING_QUEUE, stream=s2)
            ob2, _, _ = idx.join_ex(a, pending=act.ACT_PENDING_KERNEL, stream=s2)
        torch.cuda.synchronize()
        assert np.array_equal(oa.cpu().numpy(), ref_a)
        assert np.array_equal(ob.cpu().numpy(), ref_b)
        assert np.array_equal(ob2.cpu().numpy(), ref_a)


def test_overlapping_polygons_approx(act):
    P = overlapping_polygons(seed=14)
    idx = act.build(P, "approx", 2.0)
    rng = np.random.default_rng(15)
    pts = np.stack([rng.uniform(40.68, 40.72, 100000), rng.uniform(-73.98, -73.92, 100000)], 1)
    out, pairs, _ = gpu_join(idx, pts)
    assert_approx(P, pts, out, pairs, 2.0, "overlap approx")


def _uneven_batches(pts_all, rng, n_batches, hi):
    """Consecutive slices of pts_all with sizes floor(exp(U(0, ln hi))), plus
    empty and one-point batches."""
    sizes = np.maximum(1, np.floor(np.exp(rng.uniform(0, np.log(hi), n_batches)))).astype(np.int64)
    sizes[::17] = 0
    sizes[5::23] = 1
    sizes = sizes[np.cumsum(sizes) <= len(pts_all)]
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    return [(int(a), int(b)) for a, b in zip(bounds[:-1], bounds[1:])]


@pytest.mark.parametrize("mode,prec", [("exact", 0.0), ("approx", 4.0)])
def test_batched_matches_oracle_and_single(act, mode, prec):
    """Uneven batches (0 .. 2e4 points) in one batched join: every batch's
    output equals the single join's and the oracle's (exact) or meets the
    approximate guarantee; completion ticks are set and ordered after the
    start tick."""
    P, idx = index(act, "c2", mode, prec)
    rng = np.random.default_rng(31)
    pts_all = synth.workload_points("c2", 0, 1_500_000)
    spans = _uneven_batches(pts_all, rng, 400, 2e4)
    dev = torch.from_numpy(pts_all).cuda()
    batches = [(dev[a:b], torch.full((b - a,), -7, dtype=torch.int32, device="cuda"))
               for a, b in spans]
    desc, total = act.batch_descriptors(batches)
    ticks = torch.zeros(len(batches) + 1, dtype=torch.int64, device="cuda")
    idx.join_batched(desc, total, ticks=ticks)
    torch.cuda.synchronize()
    assert idx.batched_ok()
    got = np.concatenate([o.cpu().numpy() for _, o in batches])
    n = spans[-1][1]
    single = idx.join(dev[:n]).cpu().numpy()
    assert np.array_equal(got, single)
    if mode == "exact":
        ref = oracle.join(P, pts_all[:n])
        assert np.array_equal(got, ref.out)
    t = ticks.cpu().numpy().view(np.uint64)
    assert t[0] > 0 and np.all(t[1:] >= t[0])
    assert act.wall_clock_hz(0) > 1e6


def test_batched_small_batches_complete_first(act):
    """Batches are laid out smallest size class first: in an uneven mix the
    smallest quarter of the batches completes well before the largest
    quarter, and every output still equals the single join's. (Approximate
    mode: batches complete as their tiles do; in exact mode with the
    resolve kernel, batches with a pending point complete after it.)"""
    P, idx = index(act, "c2", "approx", 4.0)
    rng = np.random.default_rng(33)
    n_all = 24_000_000
    pts_all = synth.workload_points("c2", 0, n_all)
    spans = _uneven_batches(pts_all, rng, 1500, 2e5)
    rng.shuffle(spans)  # input order unrelated to size
    dev = torch.from_numpy(pts_all).cuda()
    batches = [(dev[a:b], torch.full((b - a,), -7, dtype=torch.int32, device="cuda"))
               for a, b in spans]
    desc, total = act.batch_descriptors(batches)
    ticks = torch.zeros(len(batches) + 1, dtype=torch.int64, device="cuda")
    idx.join_batched(desc, total, ticks=ticks)
    torch.cuda.synchronize()
    assert idx.batched_ok()
    single = idx.join(dev).cpu().numpy()
    for (a, b), (_, o) in zip(spans, batches):
        assert np.array_equal(o.cpu().numpy(), single[a:b]), (a, b)
    t = ticks.cpu().numpy().view(np.uint64).astype(np.float64)
    done = t[1:] - t[0]
    size = np.array([b - a for a, b in spans])
    order = np.argsort(size, kind="stable")
    q = len(order) // 4
    small, large = np.median(done[order[:q]]), np.median(done[order[-q:]])
    assert small < 0.5 * large, (small, large)


def test_batched_graph_replays(act):
    """The batched join captured once into a HIP graph (through torch) and
    replayed three times, with eager joins and output clearing between the
    replays: every replay reproduces the eager result."""
    P, idx = index(act, "c2", "exact")
    rng = np.random.default_rng(32)
    pts_all = synth.workload_points("c2", 0, 800_000)
    spans = _uneven_batches(pts_all, rng, 200, 2e4)
    dev = torch.from_numpy(pts_all).cuda()
    outs = [torch.empty(b - a, dtype=torch.int32, device="cuda") for a, b in spans]
    batches = [(dev[a:b], o) for (a, b), o in zip(spans, outs)]
    desc, total = act.batch_descriptors(batches)
    ticks = torch.zeros(len(batches) + 1, dtype=torch.int64, device="cuda")
    idx.join_batched(desc, total, ticks=ticks)
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    s = torch.cuda.Stream()
    idx.batched_reserve(len(batches), total, stream=s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        idx.join_batched(desc, total, ticks=ticks)
    for rep in range(3):
        for o in outs:
            o.fill_(-9)
        other = idx.join(dev[: 50_000 * (rep + 1)])  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), rep
        assert other.shape[0] == 50_000 * (rep + 1)


def test_batched_refuses_bad_sizes(act):
    """A batch list whose sizes exceed the stated total (so the workspace)
    or are negative is refused on the GPU: nothing is written, the status
    says so."""
    P, idx = index(act, "c1", "exact")
    pts = torch.from_numpy(synth.workload_points("c1", 0, 1000)).cuda()
    out = torch.full((1000,), -9, dtype=torch.int32, device="cuda")
    desc, total = act.batch_descriptors([(pts, out)])
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        idx.join_batched(desc, 10)  # claims 10 points, the batch has 1000
        torch.cuda.synchronize()
        assert not idx.batched_ok()
        assert int((out == -9).sum()) == 1000
        bad = desc.clone()
        bad[0, 1] = -5
        idx.join_batched(bad, 1000)
        assert not idx.batched_ok()
        idx.join_batched(desc, total)
        assert idx.batched_ok()
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), idx.join(pts).cpu().numpy())


def test_autotuner_keeps_results_and_caches(act, tmp_path):
    """act_tune sweeps launch shapes on a sample, makes the fastest the
    default (outputs unchanged), and a second tune of an identical index
    takes the configuration from the cache file."""
    P = synth.workload_polygons("c2")
    idx = act.build(P, "exact")
    pts = torch.from_numpy(synth.workload_points("c2", 0, 1_000_000)).cuda()
    before = idx.join(pts).cpu().numpy()
    cache = str(tmp_path / "act_tune.txt")
    r = idx.tune(pts, cache_path=cache)
    assert r["n_configs"] >= 20 and not r["from_cache"]
    assert r["grid"] in (256, 512, 1024, 2048, 4096) and r["points_per_lane"] in (1, 2)
    assert 0 < r["best_ms"] <= r["default_ms"] * 1.0001
    after = idx.join(pts).cpu().numpy()
    assert np.array_equal(before, after)
    idx2 = act.build(P, "exact")
    r2 = idx2.tune(pts, cache_path=cache)
    assert r2["from_cache"] and r2["index_digest"] == r["index_digest"]
    assert (r2["grid"], r2["lds_levels"], r2["points_per_lane"], r2["refine"]) == \
        (r["grid"], r["lds_levels"], r["points_per_lane"], r["refine"])
    assert np.array_equal(idx2.join(pts).cpu().numpy(), before)
    assert np.array_equal(oracle.join(P, pts[:200000].cpu().numpy()).out, before[:200000])
    # a cache line that is not a valid launch (three points per lane) is
    # skipped: the tuner times the sweep instead of applying it
    bad = str(tmp_path / "act_tune_bad.txt")
    with open(bad, "w") as f:
        f.write("%x gfx950 1024 2 3 1 1\n" % r["index_digest"])
    idx3 = act.build(P, "exact")
    r3 = idx3.tune(pts, cache_path=bad)
    assert not r3["from_cache"] and r3["n_configs"] >= 20 and r3["points_per_lane"] in (1, 2)
    assert np.array_equal(idx3.join(pts).cpu().numpy(), before)


def test_server_results_same_alone_and_in_mix(act):
    """300 requests (0 .. 2e4 points) against two resident indexes (C1 exact,
    C2 approx@4m), submitted as a burst to a 4-slot server whose arena holds
    only a few requests at once: each result equals the same request joined
    alone (and the oracle, for the exact index)."""
    P1, i1 = index(act, "c1", "exact")
    P2, i2 = index(act, "c2", "approx", 4.0)
    rng = np.random.default_rng(41)
    pool = synth.workload_points("c2", 0, 2_000_000)
    srv = act.Server([i1, i2], slots=4, arena_bytes=2_000_000, max_request_points=1 << 16)
    reqs = []
    for k in range(300):
        n = 0 if k % 29 == 0 else int(np.floor(np.exp(rng.uniform(0, np.log(2e4)))))
        a = int(rng.integers(0, len(pool) - n))
        which = int(rng.integers(0, 2))
        reqs.append((which, pool[a:a + n]))
    tickets = [srv.submit(w, p, arrival=act.Server.clock()) for w, p in reqs]
    for (w, p), t in zip(reqs, tickets):
        out, tm = srv.wait(t)
        assert tm["arrival_s"] <= tm["admitted_s"] <= tm["launched_s"] <= tm["results_s"] \
            <= tm["done_s"] and tm["n"] == len(p)
        if len(p) == 0:
            continue
        alone = (i1 if w == 0 else i2).join(torch.from_numpy(p).cuda()).cpu().numpy()
        assert np.array_equal(out, alone)
        if w == 0:
            assert np.array_equal(out, oracle.join(P1, p).out)
    st = srv.stats()
    assert st["completed"] == 300 and st["failed"] == 0 and st["queued"] == 0
    # the burst queues up behind 4 slots: waiting requests for one index
    # share launches
    assert 0 < st["launches"] < 300, st
    srv.close()


def test_server_groups_keep_results_apart(act):
    """Many tiny and empty requests for two indexes submitted at once (one
    slot, so they queue): they are joined in shared launches, each result
    equals the oracle's for its own points, in its own buffer; a request
    longer than max_request_points runs alone (its join in passes)."""
    P1, i1 = index(act, "c1", "exact")
    P2, i2 = index(act, "c1", "approx", 4.0)
    pts = synth.workload_points("c1", 0, 100_000)
    srv = act.Server([i1, i2], slots=1, arena_bytes=8 << 20, max_request_points=5000)
    rng = np.random.default_rng(43)
    reqs, a = [], 0
    for k in range(400):
        n = int(rng.choice([0, 1, 2, 63, 64, 65, 700, 4999, 5000, 12345]))
        if a + n > len(pts):
            a = 0
        reqs.append((int(rng.integers(0, 2)), pts[a:a + n]))
        a += n
    tickets = [srv.submit(w, p) for w, p in reqs]
    ref1 = oracle.join(P1, pts).out
    for (w, p), t in zip(reqs, tickets):
        out, tm = srv.wait(t)
        assert len(out) == len(p) and tm["n"] == len(p)
        if len(p) == 0:
            continue
        off = int((p.ctypes.data - pts.ctypes.data) // 16)
        if w == 0:
            assert np.array_equal(out, ref1[off:off + len(p)])
        else:
            alone = i2.join(torch.from_numpy(p).cuda()).cpu().numpy()
            assert np.array_equal(out, alone)
    st = srv.stats()
    assert st["completed"] == 400 and st["failed"] == 0
    assert st["launches"] < 200, st
    srv.close()


def test_server_large_groups_share_copies(act):
    """A burst of 30,000-point requests for one index behind one slot: the
    launch groups reach about 2^20 points (16 MiB of staging), whose copies
    are cut into pieces shared with helper threads; every result equals the
    oracle's for its own points."""
    P, idx = index(act, "c1", "exact")
    pts = synth.workload_points("c1", 0, 100_000)
    ref = oracle.join(P, pts).out
    srv = act.Server([idx], slots=1, arena_bytes=64 << 20, max_request_points=1 << 20)
    rng = np.random.default_rng(44)
    starts = rng.integers(0, len(pts) - 30_000, 96)
    tickets = [srv.submit(0, pts[a:a + 30_000]) for a in starts]
    for a, t in zip(starts, tickets):
        out, _ = srv.wait(t)
        assert np.array_equal(out, ref[a:a + 30_000]), a
    st = srv.stats()
    assert st["completed"] == 96 and st["failed"] == 0 and st["launches"] < 48, st
    srv.close()


def test_server_admission_by_memory(act):
    """Requests that each need most of the arena are admitted one at a time
    (memory, not slots, is the limit) and all complete; a request that can
    never fit is refused at submission."""
    P, idx = index(act, "c1", "exact")
    pts = synth.workload_points("c1", 0, 60_000)
    srv = act.Server([idx], slots=4, arena_bytes=20 * 50_000, max_request_points=1 << 16)
    ts = [srv.submit(0, pts[k * 10_000:k * 10_000 + 40_000]) for k in range(3)]
    for k, t in enumerate(ts):
        out, tm = srv.wait(t)
        assert np.array_equal(out, oracle.join(P, pts[k * 10_000:k * 10_000 + 40_000]).out)
    with pytest.raises(act.ActError):
        srv.submit(0, pts)  # 60k points need 1.2 MB > 1 MB arena
    assert srv.stats()["completed"] == 3
    srv.close()


def test_server_tiny_arenas(act):
    """Arenas too small for a warm-up group per slot (the warm-up shrinks
    to one point per slot, or is left out) still serve every request that
    fits them, with the oracle's results. The arenas hand out 256-byte
    granules (20 bytes a point), so a request fits if its rounded size
    does; one that fits only unrounded is refused at submission (it could
    never be admitted)."""
    P, idx = index(act, "c1", "exact")
    pts = synth.workload_points("c1", 0, 2_000)
    ref = oracle.join(P, pts).out
    for arena in (1000, 1100, 4096):
        srv = act.Server([idx], slots=4, arena_bytes=arena, max_request_points=1 << 16)
        fit = arena // 256 * 256 // 20  # 38, 51 and 204 points
        sizes = [0, 1, 5, fit]
        ts = [(k * 100, m, srv.submit(0, pts[k * 100:k * 100 + m])) for k, m in enumerate(sizes)]
        for a, m, t in ts:
            out, _ = srv.wait(t)
            assert np.array_equal(out, ref[a:a + m]), (arena, m)
        assert srv.stats()["completed"] == len(sizes)
        if arena == 1000:  # 50 points: 1000 bytes, 1024 rounded
            with pytest.raises(act.ActError):
                srv.submit(0, pts[:50])
        srv.close()


def test_server_replay_wraps_its_ring(act):
    """act_server_replay over a ring barely longer than the longest request:
    the outputs wrap around the ring and requests wait for room, and every
    request completes with a latency of at least its queueing; a request
    longer than the ring is refused before anything is submitted."""
    P, idx = index(act, "c1", "exact")
    pool = np.ascontiguousarray(synth.workload_points("c1", 0, 200_000))
    srv = act.Server([idx], slots=2, arena_bytes=8 << 20, max_request_points=1 << 16)
    rng = np.random.default_rng(17)
    n = 400
    sizes = rng.integers(0, 5000, n)
    sizes[::37] = 5000
    starts = rng.integers(0, len(pool) - 5000, n)
    arrival = act.Server.clock() + 0.01 + np.cumsum(rng.exponential(1e-5, n))
    tm = srv.replay(np.zeros(n, np.int32), [pool.ctypes.data], starts, sizes, arrival,
                    ring_points=7000)
    assert np.array_equal(tm["n"], sizes)
    assert np.all(tm["arrival_s"] == arrival)
    assert np.all(tm["admitted_s"] >= tm["arrival_s"])
    assert np.all(tm["launched_s"] >= tm["admitted_s"]) and np.all(tm["results_s"] >= tm["launched_s"])
    assert np.all(tm["done_s"] >= tm["results_s"])
    st = srv.stats()
    assert st["completed"] == n and st["failed"] == 0
    with pytest.raises(act.ActError):
        srv.replay(np.zeros(1, np.int32), [pool.ctypes.data], [0], [5000], [0.0],
                   ring_points=4000)
    assert srv.stats()["submitted"] == n
    srv.close()


def c3_sample(n_first, windows, win, seed):
    """The first n_first points of the C3 stream (batch 0) plus `windows`
    seeded windows of `win` points anywhere in its 1e9 points (60 batches)."""
    parts = [synth.workload_points("c3", 0, n_first)]
    rng = np.random.default_rng(seed)
    N = synth.WORKLOADS["c3"]["n_points"]
    for s in rng.integers(0, N - win, windows):
        parts.append(synth.workload_points("c3", int(s), int(s) + win))
    return np.concatenate(parts)


@pytest.mark.timeout(600)
def test_c3_exact_sample_all_refine_modes(act):
    """40,000 polygons, exact mode: batch-0 points and windows across the
    whole stream, every refinement mode bit-exact against the oracle."""
    P, idx = index(act, "c3", "exact")
    pts = np.concatenate([c3_sample(60_000, 16, 4096, 51),
                          edge_case_points(P, np.random.default_rng(52))[:20_000]])
    for mode in REFINE_MODES:
        out, pairs, _ = gpu_join(idx, pts, refine=getattr(act, mode))
        assert_exact(P, pts, out, pairs, "c3-" + mode)


@pytest.mark.timeout(900)
def test_c3_approx_1m_guarantee(act):
    """40,000 polygons at 1 m precision (a 3.5 GB trie, node entries read
    through 32-bit buffer offsets): no covering pair missing, every extra
    pair within 1 m of the polygon's boundary."""
    P = synth.workload_polygons("c3")
    idx = act.build(P, "approx", 1.0)
    assert idx.stats()["max_cell_level"] >= 23
    pts = c3_sample(40_000, 8, 4096, 53)
    out, pairs, _ = gpu_join(idx, pts)
    n_extra, n_pairs = assert_approx(P, pts, out, pairs, 1.0, "c3-approx1m")
    assert n_extra < 0.05 * n_pairs
    del idx


@pytest.mark.timeout(1200)
@pytest.mark.skipif(os.environ.get("ACT_SLOW_TESTS") != "1",
                    reason="builds a 7 GB trie (about 2 minutes); set ACT_SLOW_TESTS=1")
def test_c3_approx_trie_over_4gib(act):
    """40,000 polygons at 0.6 m precision: the trie's entries span more than
    4 GiB, so the probe reads them with 64-bit addresses; the approximate
    guarantee holds on the C3 sample, and the join is identical at every
    LDS depth and both point counts per lane."""
    P = synth.workload_polygons("c3")
    idx = act.build(P, "approx", 0.6)
    assert idx.stats()["node_bytes"] > (1 << 32)
    pts = c3_sample(40_000, 8, 4096, 53)
    out, pairs, _ = gpu_join(idx, pts)
    assert_approx(P, pts, out, pairs, 0.6, "c3-approx0.6")
    t = torch.from_numpy(pts).cuda()
    ref = idx.join(t)
    for lds in (0, 1, 2):
        for np_ in (1, 2):
            try:
                o, _, _ = idx.join_ex(t, lds_levels=lds, points_per_lane=np_)
            except act.ActError as e:  # top levels larger than the LDS budget
                assert e.code == -7 and lds > 0
                continue
            assert torch.equal(o, ref), (lds, np_)
    del idx


# ----------------------------------------------------- tuned launch paths

def set_launch(act, idx, path, grid, lds, np_, refine, pending):
    """Make (grid, LDS depth, points per lane, refinement, pending mode) the
    index's launch configuration through a tuning-cache line, as act_tune
    would after choosing it."""
    with open(path, "w") as f:
        f.write("%016x gfx950 %d %d %d %d %d\n" % (idx.digest(), grid, lds, np_, refine, pending))
    sample = torch.from_numpy(synth.workload_points("c1", 0, 1024)).cuda()
    r = idx.tune(sample, cache_path=str(path))
    assert r["from_cache"] == 1
    assert (r["grid"], r["lds_levels"], r["points_per_lane"], r["refine"], r["pending"]) == \
        (grid, lds, np_, refine, pending)


def run_batched(act, idx, dev, spans, stream=None):
    outs = [torch.full((b - a,), -7, dtype=torch.int32, device="cuda") for a, b in spans]
    desc, total = act.batch_descriptors([(dev[a:b], o) for (a, b), o in zip(spans, outs)])
    ticks = torch.zeros(len(spans) + 1, dtype=torch.int64, device="cuda")
    idx.join_batched(desc, total, ticks=ticks, stream=stream)
    torch.cuda.synchronize()
    assert idx.batched_ok(stream=stream)
    t = ticks.cpu().numpy().view(np.uint64)
    assert t[0] > 0 and np.all(t[1:] >= t[0])
    return outs


def test_batched_every_tuned_launch(act, tmp_path):
    """Batched joins in every launch configuration act_tune can pick (exact:
    pending points resolved by the mask's kernel or in the probe's queues,
    one or two points per lane, LDS depth 0-2, several grids; approximate:
    points per lane x LDS depth): every batch's output equals the oracle's
    (exact) or the single join's (approximate)."""
    P, idx = index(act, "c2", "exact")
    rng = np.random.default_rng(61)
    pts_all = synth.workload_points("c2", 0, 1_200_000)
    spans = _uneven_batches(pts_all, rng, 300, 2e4)
    n = spans[-1][1]
    ref = oracle.join(P, pts_all[:n]).out
    dev = torch.from_numpy(pts_all).cuda()
    grids = [256, 512, 1024, 2048, 4096]
    k = 0
    for pending in (act.ACT_PENDING_KERNEL, act.ACT_PENDING_QUEUE):
        for np_ in (1, 2):
            for lds in (0, 1, 2):
                g = grids[k % len(grids)]
                k += 1
                print("batched exact pending=%d np=%d lds=%d grid=%d" % (pending, np_, lds, g),
                      flush=True)
                set_launch(act, idx, tmp_path / "l.txt", g, lds, np_, act.ACT_REFINE_LOCAL,
                           pending)
                outs = run_batched(act, idx, dev, spans)
                got = np.concatenate([o.cpu().numpy() for o in outs])
                bad = np.nonzero(got != ref)[0]
                assert bad.size == 0, (pending, np_, lds, g, bad[:5])
    Pa, ia = index(act, "c2", "approx", 4.0)
    single = ia.join(dev[:n]).cpu().numpy()
    for np_ in (1, 2):
        for lds in (0, 1, 2):
            print("batched approx np=%d lds=%d" % (np_, lds), flush=True)
            set_launch(act, ia, tmp_path / "la.txt", 2048, lds, np_, act.ACT_REFINE_LOCAL,
                       act.ACT_PENDING_KERNEL)
            got = np.concatenate([o.cpu().numpy() for o in run_batched(act, ia, dev, spans)])
            assert np.array_equal(got, single), (np_, lds)
    # the indexes are shared with other tests: back to the built-in defaults
    for x in (idx, ia):
        set_launch(act, x, tmp_path / "d.txt", 1024, -1, 2, act.ACT_REFINE_LOCAL,
                   act.ACT_PENDING_KERNEL)


@pytest.mark.timeout(900)
def test_c4_batches_on_c3_index(act):
    """The C4 configuration: 10,000 batches of floor(exp(U(0, ln 1e6)))
    points (seed 3004) of the C3 stream against the 40,000-polygon exact
    index, in one batched join, with pending points resolved in the probe's
    queues (the autotuner's pick for this workload) and by the mask's
    kernel. The two agree on every point; the oracle checks 1% of the
    batches (seeded) and every batch under 1,000 points."""
    P, idx = index(act, "c3", "exact")
    sizes = synth.batch_sizes(10_000, 3004)
    total = int(sizes.sum())
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    print("c4: staging %d points" % total, flush=True)
    dev = torch.empty((total, 2), dtype=torch.float64, device="cuda")
    step = 1 << 24
    for s0 in range(0, total, step):
        s1 = min(total, s0 + step)
        dev[s0:s1].copy_(torch.from_numpy(synth.workload_points("c3", s0, s1)))
    spans = list(zip(bounds[:-1].tolist(), bounds[1:].tolist()))
    import tempfile
    outs = {}
    with tempfile.TemporaryDirectory() as td:
        for pending in (act.ACT_PENDING_QUEUE, act.ACT_PENDING_KERNEL):
            print("c4: pending=%d" % pending, flush=True)
            set_launch(act, idx, os.path.join(td, "c4.txt"), 256, 2, 2, act.ACT_REFINE_LOCAL,
                       pending)
            outs[pending] = run_batched(act, idx, dev, spans)
        set_launch(act, idx, os.path.join(td, "d.txt"), 1024, -1, 2, act.ACT_REFINE_LOCAL,
                   act.ACT_PENDING_KERNEL)
    for a, b in zip(outs[act.ACT_PENDING_QUEUE], outs[act.ACT_PENDING_KERNEL]):
        assert torch.equal(a, b)
    rng = np.random.default_rng(3005)
    pick = set(rng.choice(len(spans), len(spans) // 100, replace=False).tolist())
    pick |= set(np.nonzero(sizes < 1000)[0].tolist())
    pick = sorted(pick)
    print("c4: oracle on %d batches, %d points" % (len(pick), int(sizes[pick].sum())),
          flush=True)
    sel = np.concatenate([np.arange(*spans[b]) for b in pick])
    ref = oracle.join(P, dev[torch.from_numpy(sel).cuda()].cpu().numpy()).out
    got = np.concatenate([outs[act.ACT_PENDING_QUEUE][b].cpu().numpy() for b in pick])
    bad = np.nonzero(got != ref)[0]
    assert bad.size == 0, (bad.size, sel[bad[:5]])
    del dev


def test_server_with_c3_exact_index(act):
    """Serving over the two indexes of the C5 configuration (C2 approx@4m,
    C3 exact): 300 requests of 1 .. 2e4 points submitted as a burst to a
    4-slot server; every result equals the request joined alone, and the
    C3-exact results equal the oracle's."""
    P2, ia = index(act, "c2", "approx", 4.0)
    P3, ie = index(act, "c3", "exact")
    rng = np.random.default_rng(45)
    pools = [synth.workload_points("c2", 0, 1_000_000), synth.workload_points("c3", 0, 1_000_000)]
    srv = act.Server([ia, ie], slots=4, arena_bytes=4_000_000, max_request_points=1 << 16)
    reqs = []
    for k in range(300):
        n = int(np.floor(np.exp(rng.uniform(0, np.log(2e4)))))
        w = int(rng.integers(0, 2))
        a = int(rng.integers(0, len(pools[w]) - n))
        reqs.append((w, pools[w][a:a + n]))
    tickets = [srv.submit(w, p, arrival=act.Server.clock()) for w, p in reqs]
    exact_pts, exact_out = [], []
    for (w, p), t in zip(reqs, tickets):
        out, tm = srv.wait(t)
        assert tm["n"] == len(p)
        alone = (ia if w == 0 else ie).join(torch.from_numpy(p).cuda()).cpu().numpy()
        assert np.array_equal(out, alone)
        if w == 1:
            exact_pts.append(p)
            exact_out.append(out)
    ref = oracle.join(P3, np.concatenate(exact_pts)).out
    assert np.array_equal(np.concatenate(exact_out), ref)
    st = srv.stats()
    assert st["completed"] == 300 and st["failed"] == 0
    srv.close()


@pytest.mark.timeout(900)
def test_c3_exact_pin_sample(act):
    """C3 exact at the pinned sample size: the first 1e6 points of batch 0
    plus 1e6 seeded random positions of the 1e9-point stream (drawn within 64
    seeded 2^20-point chunks spread over all 60 batches), bit-exact against
    the oracle, with the pair sets."""
    P, idx = index(act, "c3", "exact")
    rng = np.random.default_rng(54)
    N = synth.WORKLOADS["c3"]["n_points"]
    chunk = 1 << 20
    parts = [synth.workload_points("c3", 0, 1_000_000)]
    for c in np.sort(rng.choice(N // chunk, 64, replace=False)):
        pts = synth.workload_points("c3", int(c) * chunk, int(c + 1) * chunk)
        parts.append(pts[np.sort(rng.choice(chunk, 1_000_000 // 64 + 1, replace=False))])
    pts = np.concatenate(parts)[:2_000_000]
    out, pairs, _ = gpu_join(idx, pts)
    assert_exact(P, pts, out, pairs, "c3-pin")


def _cell_corner_points(P, rng, n, levels):
    """Points within a few ulps of cell corners and cell edges at the given
    quadtree levels, in the cells met by polygon edges: a point on a random
    polygon edge gives a cell; its corners (and edge midpoints) are mapped
    back to lat/lng by inverting the projection, then moved by -2 .. 2 ulps
    in each coordinate."""
    v = P.verts
    a = rng.integers(0, len(v) - 1, n)
    t = rng.uniform(0, 1, (n, 1))
    on_edge = v[a] + t * (v[a + 1] - v[a])
    face, _, _, s, tt = C.project(on_edge[:, 0], on_edge[:, 1])
    i, j = C.leaf_ij(s, tt)
    lvl = rng.choice(levels, n)
    sh = 30 - lvl
    # corner offsets: 0 or 1 cell in each axis, or half a cell along an edge
    oi = rng.choice([0.0, 1.0, 0.5], n)
    oj = np.where(oi == 0.5, rng.choice([0.0, 1.0], n), rng.choice([0.0, 1.0, 0.5], n))
    si = (((i >> sh) + oi) * (2.0 ** sh)) / C.N
    sj = (((j >> sh) + oj) * (2.0 ** sh)) / C.N
    u, w = C.uv_from_st(si), C.uv_from_st(sj)
    ax = face % 3
    sign = np.where(face >= 3, -1.0, 1.0)
    c = np.zeros((3, n))
    k = np.arange(n)
    c[ax, k] = sign
    c[(ax + 1) % 3, k] = u
    c[(ax + 2) % 3, k] = w
    lat = np.degrees(np.arctan2(c[2], np.hypot(c[0], c[1])))
    lng = np.degrees(np.arctan2(c[1], c[0]))
    pts = np.stack([lat, lng], 1)
    return pts + rng.integers(-2, 3, (n, 2)) * np.spacing(pts)


@pytest.mark.parametrize("w", ["c2", "c3"])
def test_points_at_cell_edges(act, w):
    """Points within rounding of cell corners and edges at the covering's
    levels (reading: the cell boxes' 1e-9 degree margin absorbs the
    difference between the GPU's projection and any other): exact parity
    with the oracle, pairs included, in every refinement mode."""
    P, idx = index(act, w, "exact")
    st = idx.stats()
    top = st["max_cell_level"]
    pts = _cell_corner_points(P, np.random.default_rng(71), 150_000,
                              np.arange(max(1, top - 6), top + 1))
    ids = C.cell_ids(pts[:, 0], pts[:, 1])
    assert len(np.unique(ids)) > 50_000
    for mode in REFINE_MODES:
        out, pairs, _ = gpu_join(idx, pts, refine=getattr(act, mode))
        assert_exact(P, pts, out, pairs, "%s-cell-edges-%s" % (w, mode))


# ------------------------------------------------------------ trained indexes

@pytest.mark.timeout(900)
@pytest.mark.parametrize("w,n_train,max_level", [("c2", 1_000_000, 20), ("c2", 300_000, 16),
                                                 ("c3", 1_000_000, 20)])
def test_trained_index_exact(act, w, n_train, max_level):
    """Indexes trained with points of the workload's distribution (Section
    III-D; cells split below the covering level where training points hit
    candidates) stay bit-exact against the oracle in every refinement mode:
    workload points, training points (which lie in the split cells), edge
    cases and points at the corners of the trained cells."""
    P = synth.workload_polygons(w)
    tp = synth.training_points(w, n_train)
    idx = act.build(P, "exact", max_level=max_level, train_points=tp)
    st = idx.stats()
    assert st["train_splits"] > 0 and st["max_cell_level"] > max_level
    rng = np.random.default_rng(91)
    pts = np.concatenate([synth.workload_points(w, 0, 100_000), tp[:50_000],
                          edge_case_points(P, rng)[:20_000],
                          _cell_corner_points(P, rng, 30_000,
                                              np.arange(max_level, st["max_cell_level"] + 1))])
    for mode in REFINE_MODES:
        out, pairs, _ = gpu_join(idx, pts, refine=getattr(act, mode))
        assert_exact(P, pts, out, pairs, "%s-trained-%s" % (w, mode))
    # the trained index's count join agrees with its pairs
    t = torch.from_numpy(pts).cuda()
    cnt = idx.join_count(t).cpu().numpy()
    ref = oracle.join(P, pts)
    assert np.array_equal(cnt, np.bincount(ref.pair_set()[:, 1], minlength=P.n_polys))


def test_saved_and_auto_indexes(act, tmp_path):
    """An index written with act_save and read back with act_load joins
    exactly like the original (which keeps its tuned launch); ACT_AUTO
    indexes, approximate under a large budget and exact and trained under
    a smaller one, meet their modes' bars against the oracle."""
    P = synth.workload_polygons("c2")
    tp = synth.training_points("c2", 200_000)
    idx = act.build(P, "exact", train_points=tp)
    set_launch(act, idx, tmp_path / "q.txt", 512, 2, 1, act.ACT_REFINE_LOCAL,
               act.ACT_PENDING_QUEUE)
    path = tmp_path / "c2.act"
    idx.save(path)
    got = act.load(path)
    assert got.digest() == idx.digest()
    pts = np.concatenate([synth.workload_points("c2", 0, 400_000),
                          edge_case_points(P, np.random.default_rng(93))])
    t = torch.from_numpy(pts).cuda()
    a, b = idx.join(t).cpu().numpy(), got.join(t).cpu().numpy()
    assert np.array_equal(a, b)
    out, pairs, _ = gpu_join(got, pts)
    assert_exact(P, pts, out, pairs, "c2-loaded")
    approx = act.build(P, "approx", 4.0, device=-1).stats()["image_bytes"]
    big = act.build(P, "auto", 4.0, memory_budget=approx, train_points=tp)
    assert big.mode == act.ACT_APPROX
    out, pairs, _ = gpu_join(big, pts[:200_000])
    assert_approx(P, pts[:200_000], out, pairs, 4.0, "c2-auto-approx")
    small = act.build(P, "auto", 4.0, memory_budget=approx - 1, train_points=tp)
    assert small.mode == act.ACT_EXACT and small.stats()["device_bytes"] <= approx - 1
    out, pairs, _ = gpu_join(small, pts)
    assert_exact(P, pts, out, pairs, "c2-auto-exact")


@pytest.mark.parametrize("w,n_train", [("c1", 0), ("c2", 0), ("c2", 1_000_000)])
def test_budgeted_covering_exact(act, w, n_train):
    """The paper's covering configuration (per-polygon coverings of at most
    128 cells up to level 30 and 256 interior cells up to level 20, merged),
    untrained and trained: bit-exact against the oracle in every refinement
    mode, pairs included."""
    P = synth.workload_polygons(w)
    kw = {"train_points": synth.training_points(w, n_train)} if n_train else {}
    idx = act.build(P, "exact", max_level=30, max_covering_cells=128, **kw)
    st = idx.stats()
    assert st["max_cell_level"] > 20
    rng = np.random.default_rng(95)
    pts = np.concatenate([synth.workload_points(w, 0, 200_000), edge_case_points(P, rng),
                          _cell_corner_points(P, rng, 30_000,
                                              np.arange(8, st["max_cell_level"] + 1))])
    for mode in REFINE_MODES:
        out, pairs, _ = gpu_join(idx, pts, refine=getattr(act, mode))
        assert_exact(P, pts, out, pairs, "%s-budget-%d-%s" % (w, n_train, mode))


@pytest.mark.timeout(600)
@pytest.mark.parametrize("w", ["c2", "c3"])
def test_benchmark_covering_level_exact(act, w):
    """The benchmarks' exact indexes (finest covering level 22, which fills
    the deepest trie node level): bit-exact against the oracle on workload
    points, edge cases and points at cell corners down to level 22, in every
    refinement mode."""
    P = synth.workload_polygons(w)
    idx = act.build(P, "exact", max_level=22)
    assert idx.stats()["max_cell_level"] == 22
    rng = np.random.default_rng(97)
    pts = np.concatenate([synth.workload_points(w, 0, 200_000), edge_case_points(P, rng)[:20_000],
                          _cell_corner_points(P, rng, 40_000, np.arange(16, 23))])
    for mode in REFINE_MODES:
        out, pairs, _ = gpu_join(idx, pts, refine=getattr(act, mode))
        assert_exact(P, pts, out, pairs, "%s-level22-%s" % (w, mode))
