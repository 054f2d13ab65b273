"""GPU parity of the spherical geometry (ACT_GEOM_SPHERE: great-circle edges)
against the oracle's spherical model.

The sign tests use fp64 unit vectors that the GPU (table-based sin/cos) and
the oracle (C library) compute differently, so the bar is: every (point,
polygon) pair on which the two disagree has its point within 1e-6 m of that
polygon's boundary (great-circle distance); everything farther away is
identical. A rectangle with long east-west edges puts points between the
arcs and their chords, where the planar model answers differently, so the
spherical path is what decides there.
"""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def act():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_09488_amd as act
    return act


def pair_set(out, pairs):
    got = set(map(tuple, pairs.tolist())) if pairs is not None else set()
    return got | {(i, int(o)) for i, o in enumerate(out) if o >= 0}


def assert_sphere(P, pts, out, pairs, label, tol_m=1e-6):
    ref = oracle.join_sphere(P, pts)
    want = set(map(tuple, ref.pair_set().tolist()))
    got = pair_set(out, pairs)
    diff = np.asarray(sorted(got ^ want), dtype=np.int64).reshape(-1, 2)
    if len(diff):
        d = oracle.boundary_dist_sphere_pairs(P, pts, diff)
        assert d.max() <= tol_m, "%s: %d pairs differ, one %.3g m from the boundary" % (
            label, len(diff), d.max())
    return ref


def rect_polys():
    """Two rectangles sharing a long east-west edge, and one far north."""
    a = np.array([[40.0, -75.0], [40.0, -73.0], [41.0, -73.0], [41.0, -75.0]])
    b = np.array([[41.0, -75.0], [41.0, -73.0], [42.0, -73.0], [42.0, -75.0]])
    c = np.array([[44.0, -70.0], [44.0, -66.0], [45.0, -66.0], [45.0, -70.0]])
    return synth.Polygons.from_rings([[a], [b], [c]])


def bulge_points(rng, n):
    """Points spread over the rectangles, many between arcs and chords."""
    lng = rng.uniform(-75.0, -73.0, n)
    base = rng.choice([40.0, 41.0, 42.0], n)
    lat = base + rng.uniform(-0.001, 0.01, n)
    far = np.stack([rng.uniform(39.5, 45.5, n // 4), rng.uniform(-76.0, -65.0, n // 4)], 1)
    return np.concatenate([np.stack([lat, lng], 1), far])


def gpu_join(idx, pts, **kw):
    t = torch.from_numpy(np.ascontiguousarray(pts)).cuda()
    out, pairs, _ = idx.join_ex(t, capacity=max(4096, len(pts) // 4), **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy(), pairs.cpu().numpy()


def test_sphere_rectangles_between_arcs_and_chords(act):
    P = rect_polys()
    idx = act.build(P, "exact", geometry="sphere")
    pts = bulge_points(np.random.default_rng(101), 200_000)
    for refine in (act.ACT_REFINE_LOCAL, act.ACT_REFINE_FP64):
        for pending in (act.ACT_PENDING_KERNEL, act.ACT_PENDING_QUEUE):
            out, pairs = gpu_join(idx, pts, refine=refine, pending=pending)
            ref = assert_sphere(P, pts, out, pairs, "rect-%d-%d" % (refine, pending))
    # the planar model answers differently for many of these points
    plane = oracle.join(P, pts).out
    assert (plane != ref.out).sum() > 1000


@pytest.mark.parametrize("w,n", [("c1", 100_000), ("c2", 500_000)])
def test_sphere_workloads(act, w, n):
    P = synth.workload_polygons(w)
    idx = act.build(P, "exact", geometry="sphere")
    rng = np.random.default_rng(102)
    v = P.verts[rng.choice(len(P.verts), min(len(P.verts), 5000), replace=False)]
    pts = np.concatenate([synth.workload_points(w, 0, n), v,
                          v + rng.integers(-2, 3, v.shape) * np.spacing(v)])
    out, pairs = gpu_join(idx, pts)
    ref = assert_sphere(P, pts, out, pairs, w + "-sphere")
    # the other paths: count join, precomputed ids, batched
    t = torch.from_numpy(pts).cuda()
    cnt = idx.join_count(t).cpu().numpy()
    allp = np.concatenate([out[out >= 0], pairs[:, 1]])
    assert np.array_equal(cnt, np.bincount(allp, minlength=P.n_polys))
    ids = act.cell_ids(t)
    assert np.array_equal(idx.join_ids(ids, t).cpu().numpy(), out)
    half = len(pts) // 2
    outs = [torch.full((half,), -7, dtype=torch.int32, device="cuda"),
            torch.full((len(pts) - half,), -7, dtype=torch.int32, device="cuda")]
    desc, total = act.batch_descriptors([(t[:half], outs[0]), (t[half:], outs[1])])
    idx.join_batched(desc, total)
    torch.cuda.synchronize()
    assert np.array_equal(torch.cat(outs).cpu().numpy(), out)
