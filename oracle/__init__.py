"""Oracle for the point/polygon join -- TEST INFRASTRUCTURE ONLY.

Only tests, the smoke check and the benchmark's CPU-baseline leg use this
package. It is a brute-force CPU join (oracle.c) plus a numpy cell-id
reference (cellid.py); neither shares code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (OpenMP, no FMA contraction)."""
    if force or not os.path.exists(_SO):
        src = os.path.join(_HERE, "oracle.c")
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off",
                               "-fPIC", "-shared", "-Wall", "-o", tmp, src, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        d, i32, i64, p = ctypes.c_double, ctypes.c_int32, ctypes.c_int64, ctypes.c_void_p
        lib.oracle_orient_sign.argtypes = [d] * 6
        lib.oracle_orient_sign.restype = ctypes.c_int
        lib.oracle_orient_sign_exact.argtypes = [d] * 6
        lib.oracle_orient_sign_exact.restype = ctypes.c_int
        lib.oracle_orient_sign_n.argtypes = [p, i64, ctypes.c_int, p]
        lib.oracle_orient_sign_n.restype = None
        lib.oracle_covers.argtypes = [p, p, p, i32, i32, d, d, ctypes.c_int]
        lib.oracle_covers.restype = ctypes.c_int
        lib.oracle_join.argtypes = [p, p, p, i32, p, i64, p, p, p, p, i64, p,
                                    ctypes.c_int, ctypes.c_int]
        lib.oracle_join.restype = ctypes.c_int
        lib.oracle_covers_sphere.argtypes = [p, p, p, i32, i32, d, d]
        lib.oracle_covers_sphere.restype = ctypes.c_int
        lib.oracle_join_sphere.argtypes = [p, p, p, i32, p, i64, p, p, p, p, i64, p, ctypes.c_int]
        lib.oracle_join_sphere.restype = ctypes.c_int
        lib.oracle_boundary_dist_sphere_pairs.argtypes = [p, p, p, p, p, p, i64, p]
        lib.oracle_boundary_dist_sphere_pairs.restype = None
        lib.oracle_boundary_dist_m.argtypes = [p, p, p, i32, d, d]
        lib.oracle_boundary_dist_m.restype = d
        lib.oracle_boundary_dist_pairs.argtypes = [p, p, p, p, p, p, i64, p]
        lib.oracle_boundary_dist_pairs.restype = None
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _poly_args(polys):
    v = np.ascontiguousarray(polys.verts, dtype=np.float64)
    ro = np.ascontiguousarray(polys.ring_off, dtype=np.int64)
    pro = np.ascontiguousarray(polys.poly_ring_off, dtype=np.int32)
    return v, ro, pro


def orient_sign(a, b, p, exact_only: bool = False) -> int:
    """Exact sign of orient2d with points given as (x, y)."""
    f = _load().oracle_orient_sign_exact if exact_only else _load().oracle_orient_sign
    return int(f(float(a[0]), float(a[1]), float(b[0]), float(b[1]), float(p[0]), float(p[1])))


def orient_signs(abp: np.ndarray, exact_only: bool = False) -> np.ndarray:
    """Exact orientation signs of the rows (ax, ay, bx, by, px, py) of an
    (n, 6) fp64 array, as int8."""
    abp = np.ascontiguousarray(abp, dtype=np.float64).reshape(-1, 6)
    out = np.empty(abp.shape[0], np.int8)
    _load().oracle_orient_sign_n(_ptr(abp), abp.shape[0], int(exact_only), _ptr(out))
    return out


def covers(polys, p: int, lat: float, lng: float, use_bbox: bool = True) -> bool:
    v, ro, pro = _poly_args(polys)
    return bool(_load().oracle_covers(_ptr(v), _ptr(ro), _ptr(pro), polys.n_polys, int(p),
                                      float(lat), float(lng), int(use_bbox)))


class JoinResult:
    """out[i] = lowest covering polygon id or -1; cnt[i] = number of covering
    polygons; pairs = (m, 2) int64 array of the (point, polygon) pairs beyond
    out[i], sorted."""

    def __init__(self, out, cnt, pairs):
        self.out, self.cnt, self.pairs = out, cnt, pairs

    def pair_set(self) -> np.ndarray:
        """All (point, polygon) pairs, sorted, as an (m, 2) int64 array."""
        i = np.nonzero(self.out >= 0)[0]
        first = np.stack([i, self.out[i].astype(np.int64)], 1)
        allp = np.concatenate([first, self.pairs])
        order = np.lexsort((allp[:, 1], allp[:, 0]))
        return allp[order]


def join(polys, pts: np.ndarray, nthreads: int = 0, use_bbox: bool = True) -> JoinResult:
    """Brute-force join of (n, 2) fp64 (lat, lng) points against polys."""
    lib = _load()
    v, ro, pro = _poly_args(polys)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    n = pts.shape[0]
    out = np.empty(n, np.int32)
    cnt = np.empty(n, np.int32)
    cap = max(1024, n // 8)
    while True:
        pp = np.empty(cap, np.int64)
        pq = np.empty(cap, np.int32)
        m = ctypes.c_int64(0)
        lib.oracle_join(_ptr(v), _ptr(ro), _ptr(pro), polys.n_polys, _ptr(pts), n, _ptr(out),
                        _ptr(cnt), _ptr(pp), _ptr(pq), cap, ctypes.byref(m), int(nthreads),
                        int(use_bbox))
        if m.value <= cap:
            break
        cap = m.value
    m = m.value
    pairs = np.stack([pp[:m], pq[:m].astype(np.int64)], 1) if m else np.zeros((0, 2), np.int64)
    return JoinResult(out, cnt, pairs)


def covers_sphere(polys, p: int, lat: float, lng: float) -> bool:
    """Spherical model (great-circle edges): does polygon p cover the point."""
    v, ro, pro = _poly_args(polys)
    return bool(_load().oracle_covers_sphere(_ptr(v), _ptr(ro), _ptr(pro), polys.n_polys, int(p),
                                             float(lat), float(lng)))


def join_sphere(polys, pts: np.ndarray, nthreads: int = 0) -> JoinResult:
    """Brute-force join in the spherical model (great-circle edges)."""
    lib = _load()
    v, ro, pro = _poly_args(polys)
    pts = np.ascontiguousarray(pts, dtype=np.float64).reshape(-1, 2)
    n = pts.shape[0]
    out = np.empty(n, np.int32)
    cnt = np.empty(n, np.int32)
    cap = max(1024, n // 8)
    while True:
        pp = np.empty(cap, np.int64)
        pq = np.empty(cap, np.int32)
        m = ctypes.c_int64(0)
        lib.oracle_join_sphere(_ptr(v), _ptr(ro), _ptr(pro), polys.n_polys, _ptr(pts), n,
                               _ptr(out), _ptr(cnt), _ptr(pp), _ptr(pq), cap, ctypes.byref(m),
                               int(nthreads))
        if m.value <= cap:
            break
        cap = m.value
    m = m.value
    pairs = np.stack([pp[:m], pq[:m].astype(np.int64)], 1) if m else np.zeros((0, 2), np.int64)
    return JoinResult(out, cnt, pairs)


def boundary_dist_sphere_pairs(polys, pts: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """Great-circle distance in metres from each pair's point to its
    polygon's boundary (edges as minor arcs)."""
    v, ro, pro = _poly_args(polys)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    pp = np.ascontiguousarray(pairs[:, 0], dtype=np.int64)
    pq = np.ascontiguousarray(pairs[:, 1], dtype=np.int32)
    dist = np.empty(pairs.shape[0])
    _load().oracle_boundary_dist_sphere_pairs(_ptr(v), _ptr(ro), _ptr(pro), _ptr(pts), _ptr(pp),
                                              _ptr(pq), pairs.shape[0], _ptr(dist))
    return dist


def boundary_dist_m(polys, p: int, lat: float, lng: float) -> float:
    v, ro, pro = _poly_args(polys)
    return float(_load().oracle_boundary_dist_m(_ptr(v), _ptr(ro), _ptr(pro), int(p),
                                                float(lat), float(lng)))


def boundary_dist_pairs(polys, pts: np.ndarray, pairs: np.ndarray) -> np.ndarray:
    """Distance in metres from each pair's point to its polygon's boundary."""
    v, ro, pro = _poly_args(polys)
    pts = np.ascontiguousarray(pts, dtype=np.float64)
    pp = np.ascontiguousarray(pairs[:, 0], dtype=np.int64)
    pq = np.ascontiguousarray(pairs[:, 1], dtype=np.int32)
    dist = np.empty(pairs.shape[0])
    _load().oracle_boundary_dist_pairs(_ptr(v), _ptr(ro), _ptr(pro), _ptr(pts), _ptr(pp),
                                       _ptr(pq), pairs.shape[0], _ptr(dist))
    return dist
