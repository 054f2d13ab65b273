"""GPU tests of the workspace lifetime and the pair-overflow status entry
points (act_workspace_release, act_join_status) through the C ABI."""
import ctypes

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


def test_release_between_short_lived_streams(act):
    """Joins on fresh streams, each released afterwards (twice: the second
    call is a no-op), give the oracle's output every time, also when the
    stream's workspace was reserved larger first."""
    P = synth.workload_polygons("c1")
    idx = act.build(P, "exact")
    pts_np = np.concatenate([synth.workload_points("c1", 0, 50_000), P.verts])
    pts = torch.from_numpy(pts_np).cuda()
    want = oracle.join(P, pts_np).out
    for k in range(4):
        s = torch.cuda.Stream()
        if k % 2:
            idx.reserve(1 << 20, stream=s)
        with torch.cuda.stream(s):
            got = idx.join(pts)
        idx.release(stream=s)
        idx.release(stream=s)
        s.synchronize()
        assert np.array_equal(got.cpu().numpy(), want), k
    idx.release()  # the default stream holds no workspace of this index yet


def test_join_status_reports_overflow(act):
    """act_join_status: ACT_OK at or under the capacity, ACT_E_OVERFLOW above
    it, with the counter returned; a pair join with too small a capacity
    raises with the number of pairs needed, and one with that capacity
    returns the oracle's pair set."""
    from paper_1802_09488_amd import _binding as B
    cnt = torch.tensor([5], dtype=torch.int64, device="cuda")
    m = ctypes.c_int64()
    assert B.lib.act_join_status(ctypes.c_void_p(cnt.data_ptr()), 5, None, ctypes.byref(m)) == 0
    assert m.value == 5
    rc = B.lib.act_join_status(ctypes.c_void_p(cnt.data_ptr()), 4, None, ctypes.byref(m))
    assert rc == B.ACT_E_OVERFLOW and m.value == 5
    P = synth.workload_polygons("c1")
    idx = act.build(P, "exact")
    pts_np = P.verts.copy()  # shared vertices: several pairs per point
    pts = torch.from_numpy(pts_np).cuda()
    ref = oracle.join(P, pts_np)
    with pytest.raises(act.ActError) as e:
        idx.join_ex(pts, capacity=1)
    assert e.value.code == B.ACT_E_OVERFLOW and e.value.needed == len(ref.pairs)
    out, pairs, _ = idx.join_ex(pts, capacity=len(ref.pairs))
    pr = pairs.cpu().numpy()
    pr = pr[np.lexsort((pr[:, 1], pr[:, 0]))]
    assert np.array_equal(out.cpu().numpy(), ref.out)
    assert np.array_equal(pr, ref.pairs)
