"""act_join_noalloc (the join that allocates nothing) against act_join.

Calls both entry points through the C ABI on the same points and requires
identical outputs, on two calls in a row (the second smaller, so stale mask
words of the first call would show), for an exact and an approximate index,
and for an exact index whose pending points are resolved in the probe's
queues. Sizes beyond the documented limit are refused before any launch.
"""
import ctypes

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def act():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1802_09488_amd as act
    return act


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(act, idx, pts):
    """(act_join output, act_join_noalloc output) for the same points."""
    lib = act.lib
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    n = pts.shape[0]
    ref = torch.full((n,), -7, dtype=torch.int32, device=pts.device)
    got = torch.full((n,), -9, dtype=torch.int32, device=pts.device)
    rc = lib.act_join(idx.handle, _ptr(pts), n, _ptr(ref), stream)
    assert rc == 0, lib.act_last_error().decode()
    rc = lib.act_join_noalloc(idx.handle, _ptr(pts), n, _ptr(got), stream)
    assert rc == 0, lib.act_last_error().decode()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), got.cpu().numpy()


def _points(w, n0, n1):
    return torch.from_numpy(synth.workload_points(w, n0, n1)).cuda()


@pytest.mark.parametrize("w,mode,prec", [("c2", "exact", 0.0), ("c2", "approx", 4.0),
                                         ("c1", "exact", 0.0)])
def test_noalloc_matches_join_twice(act, w, mode, prec):
    idx = act.build(synth.workload_polygons(w), mode, prec)
    big = _points(w, 0, 3_000_017)
    small = _points(w, 5_000_000, 5_200_003)
    for label, pts in (("first call", big), ("second, smaller call", small)):
        print("noalloc %s %s %s n=%d" % (w, mode, label, pts.shape[0]), flush=True)
        ref, got = _both(act, idx, pts)
        bad = np.nonzero(ref != got)[0]
        assert bad.size == 0, "%s: %d outputs differ, first at %s" % (label, bad.size, bad[:5])
        if mode == "exact":
            assert (ref >= 0).mean() > 0.5


def test_noalloc_with_queue_resolve(act, tmp_path):
    # an exact index whose launch configuration resolves pending points in
    # the probe's queues (set through a tuning-cache line)
    idx = act.build(synth.workload_polygons("c1"), "exact")
    cache = tmp_path / "tune.txt"
    cache.write_text("%016x gfx950 512 2 2 1 2\n" % idx.digest())
    sample = _points("c1", 0, 4096)
    r = idx.tune(sample, cache_path=str(cache))
    assert r["from_cache"] == 1 and r["pending"] == act.ACT_PENDING_QUEUE
    for n0, n1 in ((0, 100_000), (200_000, 230_001)):
        ref, got = _both(act, idx, _points("c1", n0, n1))
        assert np.array_equal(ref, got)


def test_noalloc_refuses_beyond_limit_and_accepts_empty(act):
    idx = act.build(synth.workload_polygons("c1"), "exact")
    lib = act.lib
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    pts = _points("c1", 0, 64)
    out = torch.empty(64, dtype=torch.int32, device="cuda")
    # the size check comes before anything is launched or read
    rc = lib.act_join_noalloc(idx.handle, _ptr(pts), (1 << 27) + 1, _ptr(out), stream)
    assert rc == act._binding.ACT_E_RANGE
    assert "limit" in lib.act_last_error().decode()
    assert lib.act_join_noalloc(idx.handle, _ptr(pts), 0, _ptr(out), stream) == 0
    assert lib.act_join_noalloc(idx.handle, _ptr(pts), -1, _ptr(out), stream) == \
        act._binding.ACT_E_ARG
