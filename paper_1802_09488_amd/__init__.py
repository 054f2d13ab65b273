"""MI355X (gfx950) Adaptive Cell Trie point/polygon join.

Kipf et al., "Adaptive Geospatial Joins for Modern Hardware" (arXiv
1802.09488): polygons are approximated by a precision-preserving super
covering of cube-face/Hilbert cells stored in an Adaptive Cell Trie
(Sections III-B, III-C); streaming points are probed against it on the GPU
(Section III-E) and candidate hits are refined by an exact point-in-polygon
test. This package is a thin binding of the C ABI in include/act.h.

    idx = build(polys, mode="exact")               # host build + upload
    out = idx.join(points)                         # (n,) int32 on the GPU
    out, pairs = idx.join_pairs(points)            # all (point, polygon) pairs

`polys` is any object with .verts (V,2 float64 lat,lng), .ring_off (int64)
and .poly_ring_off (int32) in the CSR layout of act_build; `points` is an
(n, 2) float64 (lat, lng) CUDA tensor.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _binding as _b
from ._binding import (ACT_APPROX, ACT_AUTO, ACT_EXACT, ACT_PENDING_AUTO, ACT_PENDING_KERNEL,
                       ACT_PENDING_QUEUE, ACT_REFINE_AUTO, ACT_REFINE_FP32_FILTER,
                       ACT_REFINE_FP64, ACT_REFINE_LOCAL, COUNTER_NAMES, ActError)

__all__ = ["build", "load", "Index", "Server", "cell_ids", "batch_descriptors",
           "wall_clock_hz", "ActError",
           "ACT_EXACT", "ACT_APPROX", "ACT_AUTO",
           "ACT_REFINE_AUTO", "ACT_REFINE_LOCAL", "ACT_REFINE_FP32_FILTER", "ACT_REFINE_FP64",
           "ACT_PENDING_AUTO", "ACT_PENDING_KERNEL", "ACT_PENDING_QUEUE",
           "version", "lib"]

lib = _b.lib


def version() -> str:
    return lib.act_version().decode()


def _np_ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _stream_ptr(stream):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _check_points(points):
    import torch
    if not isinstance(points, torch.Tensor) or not points.is_cuda:
        raise TypeError("points must be a CUDA tensor")
    if points.dtype != torch.float64 or points.dim() != 2 or points.shape[1] != 2:
        raise TypeError("points must be an (n, 2) float64 tensor of (lat, lng)")
    if not points.is_contiguous():
        raise TypeError("points must be contiguous")


class Index:
    """A built index (host structure + HBM image). Immutable; joins on it may
    run concurrently on different streams."""

    def __init__(self, handle, mode, precision_m, device):
        self._h = handle
        self.mode = mode
        self.precision_m = precision_m
        self.device = device

    def __del__(self, _free=lib.act_free):
        h, self._h = getattr(self, "_h", None), None
        if h:
            _free(h)

    def close(self):
        self.__del__()

    @property
    def handle(self):
        return self._h

    def save(self, path):
        """Write the index (host image and launch configuration) to a file."""
        _b.check(lib.act_save(self._h, str(path).encode()))

    def stats(self) -> dict:
        st = _b.Stats()
        _b.check(lib.act_index_stats(self._h, ctypes.byref(st)))
        return st.as_dict()

    def join(self, points, out=None, stream=None):
        """out[i] = lowest matching polygon id or -1 (int32 CUDA tensor)."""
        import torch
        _check_points(points)
        n = points.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=points.device)
        _b.check(lib.act_join(self._h, ctypes.c_void_p(points.data_ptr()), n,
                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def join_ids(self, ids, points=None, out=None, stream=None):
        """Join points given by their level-30 cell ids (int64 CUDA tensor of
        the uint64 bit patterns, as cell_ids() returns); `points` (the same
        points' (n, 2) float64 lat/lng) is required in exact mode."""
        import torch
        if not isinstance(ids, torch.Tensor) or not ids.is_cuda or ids.dtype != torch.int64 \
                or ids.dim() != 1 or not ids.is_contiguous():
            raise TypeError("ids must be a contiguous 1-D int64 CUDA tensor")
        n = ids.shape[0]
        if points is not None:
            _check_points(points)
            if points.shape[0] != n:
                raise ValueError("ids and points differ in length")
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=ids.device)
        _b.check(lib.act_join_ids(self._h, ctypes.c_void_p(ids.data_ptr()),
                                  ctypes.c_void_p(points.data_ptr() if points is not None else 0),
                                  n, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def join_count(self, points, counts=None, stream=None):
        """Per-polygon number of covering points (int64 CUDA tensor of
        n_polys), added to `counts` when given (streaming), else to zeros."""
        import torch
        _check_points(points)
        if counts is None:
            counts = torch.zeros(self.n_polys, dtype=torch.int64, device=points.device)
        elif counts.dtype != torch.int64 or counts.numel() < self.n_polys or \
                not counts.is_contiguous():
            raise TypeError("counts must be a contiguous int64 tensor of n_polys elements")
        _b.check(lib.act_join_count(self._h, ctypes.c_void_p(points.data_ptr()),
                                    points.shape[0], ctypes.c_void_p(counts.data_ptr()),
                                    _stream_ptr(stream)))
        return counts

    @property
    def n_polys(self) -> int:
        return int(self.stats()["n_polys"])

    def join_ex(self, points, out=None, *, capacity=None, counters=False,
                refine=ACT_REFINE_AUTO, block=0, lds_levels=-1, grid=0,
                pass_points=0, points_per_lane=0, pending=ACT_PENDING_AUTO,
                probe_event=None, stream=None):
        """Full-control join. Returns (out, pairs or None, counters dict or None).

        pairs: (m, 2) int64 CUDA tensor of (point, polygon) beyond out[i]
        when `capacity` is given (ActError ACT_E_OVERFLOW if it was too
        small)."""
        import torch
        _check_points(points)
        n = points.shape[0]
        dev = points.device
        if out is None:
            out = torch.empty(n, dtype=torch.int32, device=dev)
        a = _b.JoinArgs()
        a.d_points = points.data_ptr()
        a.n = n
        a.d_out = out.data_ptr()
        a.refine = refine
        a.block = block
        a.lds_levels = lds_levels
        a.grid = grid
        a.pass_points = pass_points
        a.points_per_lane = points_per_lane
        a.pending = pending
        if probe_event is not None:  # a recorded torch.cuda.Event (its HIP event handle)
            a.probe_event = probe_event.cuda_event
        pp = pq = cnt = ctr = None
        if capacity is not None:
            pp = torch.empty(max(1, capacity), dtype=torch.int64, device=dev)
            pq = torch.empty(max(1, capacity), dtype=torch.int32, device=dev)
            cnt = torch.zeros(1, dtype=torch.int64, device=dev)
            a.d_pair_point, a.d_pair_poly, a.d_n_pairs = pp.data_ptr(), pq.data_ptr(), cnt.data_ptr()
            a.pair_capacity = capacity
        if counters:
            ctr = torch.zeros(_b.ACT_NCOUNTERS, dtype=torch.int64, device=dev)
            a.d_counters = ctr.data_ptr()
        _b.check(lib.act_join_ex(self._h, ctypes.byref(a), _stream_ptr(stream)))
        pairs = None
        if capacity is not None:
            m = ctypes.c_int64()
            rc = lib.act_join_status(ctypes.c_void_p(cnt.data_ptr()), int(capacity),
                                     _stream_ptr(stream), ctypes.byref(m))
            if rc == _b.ACT_E_OVERFLOW:
                err = ActError(rc, lib.act_last_error().decode())
                err.needed = m.value
                raise err
            _b.check(rc)
            pairs = torch.stack([pp[:m.value], pq[:m.value].to(torch.int64)], 1)
        cdict = None
        if counters:
            c = ctr.cpu().numpy()
            cdict = {k: int(c[i]) for i, k in enumerate(COUNTER_NAMES)}
        return out, pairs, cdict

    def reserve(self, points, stream=None):
        """Size the stream's exact-mode workspace for `points` points per pass."""
        _b.check(lib.act_workspace_reserve(self._h, _stream_ptr(stream), int(points)))

    def release(self, stream=None):
        """Free the workspaces joins on `stream` hold in this index (call
        before dropping a stream that ran joins)."""
        _b.check(lib.act_workspace_release(self._h, _stream_ptr(stream)))

    def join_batched(self, descriptors, total_points, ticks=None, stream=None):
        """Join many batches at once. `descriptors`: CUDA int64 tensor (nb, 3)
        from batch_descriptors(); `ticks`: optional CUDA int64 tensor of
        nb + 1 (GPU wall-clock ticks: start, then each batch's completion).
        Enqueues only (graph-capturable once the workspace is reserved)."""
        nb = int(descriptors.shape[0])
        _b.check(lib.act_join_batched(self._h, ctypes.c_void_p(descriptors.data_ptr()), nb,
                                      int(total_points),
                                      ctypes.c_void_p(ticks.data_ptr() if ticks is not None else 0),
                                      _stream_ptr(stream)))

    def digest(self) -> int:
        d = ctypes.c_uint64()
        _b.check(lib.act_index_digest(self._h, ctypes.byref(d)))
        return d.value

    def tune(self, sample, cache_path=None, stream=None) -> dict:
        """Autotune the launch configuration on a sample of points (CUDA
        (n, 2) float64); see act_tune. Returns the choice and timings."""
        import torch
        _check_points(sample)
        scratch = torch.empty(sample.shape[0], dtype=torch.int32, device=sample.device)
        r = _b.TuneResult()
        cp = cache_path.encode() if cache_path else None
        _b.check(lib.act_tune(self._h, ctypes.c_void_p(sample.data_ptr()), int(sample.shape[0]),
                              ctypes.c_void_p(scratch.data_ptr()), _stream_ptr(stream), cp,
                              ctypes.byref(r)))
        return {k: getattr(r, k) for k, _ in r._fields_}

    def batched_reserve(self, max_batches, max_points, stream=None):
        _b.check(lib.act_batched_reserve(self._h, _stream_ptr(stream), int(max_batches),
                                         int(max_points)))

    def batched_ok(self, stream=None) -> bool:
        ok = ctypes.c_int32(0)
        _b.check(lib.act_batched_status(self._h, _stream_ptr(stream), ctypes.byref(ok)))
        return bool(ok.value)

    def join_pairs(self, points, capacity=None, stream=None):
        """(out, pairs): pairs is (m, 2) int64 of (point, polygon) beyond out[i].
        Retries once with the exact size if the first capacity was too small."""
        n = points.shape[0]
        cap = max(1024, n // 16) if capacity is None else capacity
        try:
            out, pairs, _ = self.join_ex(points, capacity=cap, stream=stream)
        except ActError as e:
            if e.code != _b.ACT_E_OVERFLOW or capacity is not None:
                raise
            out, pairs, _ = self.join_ex(points, capacity=e.needed, stream=stream)
        return out, pairs

    def lookup_host(self, face, i, j) -> np.ndarray:
        """Host trie lookup of leaf cells (face, i, j): tagged entries."""
        f = np.ascontiguousarray(face, dtype=np.int32)
        a = np.ascontiguousarray(i, dtype=np.uint32)
        b = np.ascontiguousarray(j, dtype=np.uint32)
        ent = np.empty(f.shape[0], np.uint64)
        _b.check(lib.act_lookup_host(self._h, _np_ptr(f), _np_ptr(a), _np_ptr(b), f.shape[0],
                                     _np_ptr(ent)))
        return ent

    def refine_local_host(self, face, i, j, lat, lng, poly) -> bool:
        """Evaluate the cell-local refinement record on the host."""
        c = ctypes.c_int32(0)
        _b.check(lib.act_refine_local_host(self._h, int(face), int(i), int(j), float(lat),
                                           float(lng), int(poly), ctypes.byref(c)))
        return bool(c.value)

    def lut_host(self) -> np.ndarray:
        n = ctypes.c_int64(0)
        _b.check(lib.act_lut_host(self._h, None, ctypes.byref(n)))
        w = np.empty(n.value, np.uint32)
        _b.check(lib.act_lut_host(self._h, _np_ptr(w), ctypes.byref(n)))
        return w


def build(polys, mode="exact", precision_m: float = 0.0, *, max_level: int = 20,
          device: int = 0, threads: int = 0, margin_deg: float = 0.0,
          prefix_level: int = -1, train_points=None, memory_budget: int = 0,
          train_max_level: int = 30, geometry: str = "plane", max_covering_cells: int = 0,
          max_interior_cells: int = 256, max_interior_level: int = 20) -> Index:
    """Build an index (host) and upload it to `device` (-1: host only).
    prefix_level -1 lets the builder choose the trie's prefix level.
    train_points: optional (n, 2) float64 (lat, lng) host array the exact
    index is trained with (Section III-D) within memory_budget bytes of
    device image (0: no limit). geometry "sphere": edges are great-circle
    arcs (exact mode). max_covering_cells > 0: per-polygon coverings with
    cell budgets (the paper's configuration: 128, 256, 20 with max_level
    30) instead of the joint subdivision."""
    m = {"exact": ACT_EXACT, "approx": ACT_APPROX, "auto": ACT_AUTO}.get(mode, mode)
    v = np.ascontiguousarray(polys.verts, dtype=np.float64)
    ro = np.ascontiguousarray(polys.ring_off, dtype=np.int64)
    pro = np.ascontiguousarray(polys.poly_ring_off, dtype=np.int32)
    n_polys = pro.shape[0] - 1
    tp = None if train_points is None else \
        np.ascontiguousarray(train_points, dtype=np.float64).reshape(-1, 2)
    opts = _b.BuildOpts(max_level=max_level, device=device, threads=threads,
                        prefix_level=prefix_level, margin_deg=margin_deg,
                        train_points=tp.ctypes.data if tp is not None else None,
                        n_train=0 if tp is None else tp.shape[0],
                        memory_budget=int(memory_budget), train_max_level=train_max_level,
                        geometry={"plane": _b.ACT_GEOM_PLANE,
                                  "sphere": _b.ACT_GEOM_SPHERE}.get(geometry, geometry),
                        max_covering_cells=max_covering_cells,
                        max_interior_cells=max_interior_cells,
                        max_interior_level=max_interior_level)
    h = ctypes.c_void_p()
    _b.check(lib.act_build(_np_ptr(v), _np_ptr(ro), _np_ptr(pro), n_polys, m, float(precision_m),
                           ctypes.byref(opts), ctypes.byref(h)))
    idx = Index(h, m, precision_m, device)
    if m == ACT_AUTO:  # the mode the budget policy took
        idx.mode = idx.stats()["mode"]
    return idx


def load(path, device: int = 0) -> Index:
    """An index saved with Index.save, uploaded to `device` (-1: host only)."""
    h = ctypes.c_void_p()
    _b.check(lib.act_load(str(path).encode(), int(device), ctypes.byref(h)))
    idx = Index(h, ACT_EXACT, 0.0, device)
    st = idx.stats()
    idx.mode, idx.precision_m = st["mode"], st["precision_m"]
    return idx


def batch_descriptors(batches):
    """Device array of act_batch descriptors for [(points, out), ...] (CUDA
    tensors: points (n, 2) float64, out (n,) int32). Returns (descriptors,
    total points). The tensors must stay alive while joins use them."""
    import torch
    rows = []
    total = 0
    for pts, out in batches:
        _check_points(pts)
        n = int(pts.shape[0])
        if out.dtype != torch.int32 or out.shape[0] < n or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor of at least n elements")
        rows.append((pts.data_ptr(), n, out.data_ptr()))
        total += n
    dev = batches[0][0].device if batches else "cuda"
    d = torch.tensor(rows, dtype=torch.int64).reshape(-1, 3).to(dev)
    return d, total


class Server:
    """Serving loop over resident indexes (act_server_*): requests of host
    (n, 2) float64 points are admitted by free slots and arena memory and
    overlap on the GPU; results land in host int32 arrays."""

    def __init__(self, indexes, slots=4, arena_bytes=0, max_request_points=1 << 20, device=0):
        self._indexes = list(indexes)  # keeps them alive
        o = _b.ServerOpts()
        lib.act_server_opts_init(ctypes.byref(o))
        o.slots, o.arena_bytes, o.max_request_points, o.device = (
            slots, arena_bytes, max_request_points, device)
        arr = (ctypes.c_void_p * len(self._indexes))(*[x._h.value for x in self._indexes])
        h = ctypes.c_void_p()
        rc = lib.act_server_create(arr, len(self._indexes), ctypes.byref(o), ctypes.byref(h))
        if rc:
            raise ActError(rc, lib.act_server_last_error().decode())
        self._h = h
        self._live = {}

    @staticmethod
    def clock() -> float:
        return lib.act_server_clock()

    def submit(self, index, points, out=None, arrival=0.0):
        pts = np.ascontiguousarray(points, dtype=np.float64)
        if pts.ndim != 2 or pts.shape[1] != 2:
            raise TypeError("points must be (n, 2) float64")
        if out is None:
            out = np.empty(pts.shape[0], dtype=np.int32)
        t = ctypes.c_uint64()
        rc = lib.act_server_submit(self._h, int(index), _np_ptr(pts), pts.shape[0], _np_ptr(out),
                                   float(arrival), ctypes.byref(t))
        if rc:
            raise ActError(rc, lib.act_server_last_error().decode())
        self._live[t.value] = (pts, out)
        return t.value

    def wait(self, ticket):
        """(out, times dict) of a submitted request."""
        tm = _b.RequestTimes()
        rc = lib.act_server_wait(self._h, ctypes.c_uint64(ticket), ctypes.byref(tm))
        pts, out = self._live.pop(ticket)
        if rc:
            raise ActError(rc, lib.act_server_last_error().decode())
        return out, {k: getattr(tm, k) for k, _ in tm._fields_}

    def replay(self, index, pool_ptrs, starts, sizes, arrival, ring_points=1 << 26):
        """Native load generator (act_server_replay): request k joins
        sizes[k] points starting at row starts[k] of host pool index[k]
        (pool_ptrs[index[k]]: the address of a C-contiguous (m, 2) float64
        array the caller keeps alive) at arrival[k] (Server.clock()
        seconds). Returns a structured array of each request's arrival_s,
        admitted_s, launched_s, results_s and done_s (Server.clock()
        seconds) and n."""
        index = np.ascontiguousarray(index, dtype=np.int32)
        sizes = np.ascontiguousarray(sizes, dtype=np.int64)
        arrival = np.ascontiguousarray(arrival, dtype=np.float64)
        base = np.asarray(pool_ptrs, dtype=np.uint64)[index]
        ptrs = np.ascontiguousarray(base + 16 * np.asarray(starts, dtype=np.uint64))
        times = np.zeros(len(sizes), dtype=[("arrival_s", np.float64), ("admitted_s", np.float64),
                                            ("launched_s", np.float64), ("results_s", np.float64),
                                            ("done_s", np.float64), ("n", np.int64)])
        rc = lib.act_server_replay(self._h, len(sizes), _np_ptr(index), _np_ptr(ptrs),
                                   _np_ptr(sizes), _np_ptr(arrival), int(ring_points),
                                   _np_ptr(times))
        if rc:
            raise ActError(rc, lib.act_server_last_error().decode())
        return times

    def stats(self) -> dict:
        st = _b.ServerStats()
        _b.check(lib.act_server_stats_get(self._h, ctypes.byref(st)))
        return {k: getattr(st, k) for k, _ in st._fields_ if k != "reserved"}

    def close(self):
        if getattr(self, "_h", None):
            lib.act_server_destroy(self._h)
            self._h = None
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wall_clock_hz(device: int = 0) -> float:
    """Tick rate of the GPU wall clock behind batched-join ticks."""
    hz = ctypes.c_double(0.0)
    _b.check(lib.act_wall_clock_hz(int(device), ctypes.byref(hz)))
    return hz.value


def cell_ids(points, out=None, stream=None):
    """Level-30 cell ids (int64 CUDA tensor holding the uint64 bit patterns)."""
    import torch
    _check_points(points)
    n = points.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device=points.device)
    _b.check(lib.act_cell_ids(ctypes.c_void_p(points.data_ptr()), n,
                              ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def encode_refs_host(refs, lut=None, lut_cap=4096):
    """Encode a reference list (ids << 1 | interior) as the builder does.
    Returns (entry, lut words)."""
    r = np.ascontiguousarray(refs, dtype=np.uint32)
    buf = np.zeros(lut_cap, np.uint32)
    n = 0 if lut is None else len(lut)
    if lut is not None:
        buf[:n] = lut
    ln = ctypes.c_int64(n)
    e = ctypes.c_uint64(0)
    _b.check(lib.act_encode_refs_host(_np_ptr(r), r.shape[0], _np_ptr(buf), lut_cap,
                                      ctypes.byref(ln), ctypes.byref(e)))
    return int(e.value), buf[:ln.value].copy()


def orient_fp32_host(a, b, p, origin, m_poly) -> int:
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, p, origin)]
    return int(lib.act_orient_fp32_host(*[_np_ptr(x) for x in arr], ctypes.c_float(m_poly)))


def orient_host_n(abp, tier, origin=None, m_poly=None) -> np.ndarray:
    """Signs of the rows (ax, ay, bx, by, px, py) of an (n, 6) array by the
    library's exact tier (tier 0) or its fp32 tier (tier 1: 0 = undecided)."""
    abp = np.ascontiguousarray(abp, dtype=np.float64).reshape(-1, 6)
    n = abp.shape[0]
    out = np.empty(n, np.int8)
    o = np.ascontiguousarray(origin if origin is not None else np.zeros((n, 2)), dtype=np.float64)
    m = np.ascontiguousarray(m_poly if m_poly is not None else np.zeros(n), dtype=np.float32)
    _b.check(lib.act_orient_host_n(_np_ptr(abp), _np_ptr(o), _np_ptr(m), n, int(tier),
                                   _np_ptr(out)))
    return out


def orient_exact_host(a, b, p) -> int:
    arr = [np.ascontiguousarray(x, dtype=np.float64) for x in (a, b, p)]
    return int(lib.act_orient_exact_host(*[_np_ptr(x) for x in arr]))
