"""GPU parity of the per-polygon count join (act_join_count), the paper's
evaluation query (a count of the join pairs grouped by polygon id).

Exact mode: counts[p] equals the number of points the oracle finds covered
by polygon p (np.bincount of its pair set), overlaps and shared boundaries
included. Approximate mode: counts equal the bincount of the same index's
pair output (every reference of a point's cell), which the approximate
guarantee tests check against the oracle, and no count is below the
oracle's.
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


_IDX = {}


def index(act, w, mode, prec=0.0):
    key = (w, mode, prec)
    if key not in _IDX:
        P = synth.workload_polygons(w)
        _IDX[key] = (P, act.build(P, mode, prec))
    return _IDX[key]


def oracle_counts(P, pts):
    ref = oracle.join(P, pts)
    return np.bincount(ref.pair_set()[:, 1], minlength=P.n_polys).astype(np.int64)


def edge_points(P, rng, n=4000):
    v = P.verts
    k = rng.choice(len(v), min(len(v), n), replace=False)
    nudged = v[k] + rng.integers(-1, 2, (len(k), 2)) * np.spacing(v[k])
    bad = np.array([[np.nan, -74.0], [91.0, -74.0], [40.7, 106.0]])
    mids = 0.5 * (v[:-1] + v[1:])
    return np.concatenate([v[k], nudged, mids[k[k < len(mids)]], bad])


@pytest.mark.parametrize("w,n", [("c1", 100_000), ("c2", 1_000_000), ("c3", 200_000)])
def test_count_exact_matches_oracle(act, w, n):
    P, idx = index(act, w, "exact")
    pts = np.concatenate([synth.workload_points(w, 0, n), edge_points(P, np.random.default_rng(81))])
    got = idx.join_count(torch.from_numpy(pts).cuda()).cpu().numpy()
    want = oracle_counts(P, pts)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, (w, bad[:5], got[bad[:5]], want[bad[:5]])
    assert got.sum() >= (want > 0).sum()


@pytest.mark.parametrize("w,prec", [("c1", 4.0), ("c2", 4.0)])
def test_count_approx_matches_pairs(act, w, prec):
    P, idx = index(act, w, "approx", prec)
    pts = synth.workload_points(w, 0, 1_000_000)
    t = torch.from_numpy(pts).cuda()
    got = idx.join_count(t).cpu().numpy()
    out, pairs = idx.join_pairs(t)
    out = out.cpu().numpy()
    allp = np.concatenate([out[out >= 0], pairs[:, 1].cpu().numpy()]) if pairs is not None \
        else out[out >= 0]
    assert np.array_equal(got, np.bincount(allp, minlength=P.n_polys))
    assert np.all(got >= oracle_counts(P, pts))


def test_count_accumulates_and_handles_small_inputs(act):
    """Counts add up over calls (a stream in chunks equals one call), for
    ragged chunk sizes from 0 to a few tiles, in both modes and with the
    resolve kernel's lists and the LDS histogram."""
    for mode, prec in (("exact", 0.0), ("approx", 4.0)):
        P, idx = index(act, "c2", mode, prec)
        pts = torch.from_numpy(synth.workload_points("c2", 0, 300_000)).cuda()
        whole = idx.join_count(pts)
        acc = torch.zeros_like(whole)
        cuts = [0, 0, 1, 2, 63, 64, 65, 127, 128, 129, 4095, 70_000, 300_000]
        for a, b in zip(cuts[:-1], cuts[1:]):
            idx.join_count(pts[a:b], counts=acc)
        torch.cuda.synchronize()
        assert torch.equal(whole, acc), mode


def test_count_c3_full_batch_vs_pairs(act):
    """A whole 2^24-point C3 batch (global counters: 40,000 polygons do not
    fit the LDS histogram) equals the bincount of the exact pair output."""
    P, idx = index(act, "c3", "exact")
    pts = torch.from_numpy(synth.workload_points("c3", 0, 1 << 24)).cuda()
    got = idx.join_count(pts).cpu().numpy()
    out, pairs = idx.join_pairs(pts)
    out = out.cpu().numpy()
    allp = np.concatenate([out[out >= 0], pairs[:, 1].cpu().numpy()])
    assert np.array_equal(got, np.bincount(allp, minlength=P.n_polys))
