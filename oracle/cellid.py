"""Reference cell ids -- TEST INFRASTRUCTURE ONLY (numpy, fp64).

Section "Background" (Google S2 paragraph) describes the discretisation: a
point on the sphere is projected onto the surrounding unit cube, each of the
six faces is split recursively as a quadtree, and cells are numbered in
Hilbert order as 64-bit ids: 3 face bits, then one bit pair per level
(0..30 of them), then a set marker bit, then zeros. The paper fixes neither
the face numbering, the (u, v) axes, the uv->st transform nor the curve's
orientation, and requires only that a child's id extends its parent's prefix
(Section "Background", space-filling curves paragraph). The reading used by
this project:

  * x = cos(lat) cos(lng), y = cos(lat) sin(lng), z = sin(lat);
  * axis a = argmax(|x|, |y|, |z|), ties to the lower axis;
    face = a (positive side) or a + 3 (negative side);
  * u = c[(a+1) % 3] / |c[a]|, v = c[(a+2) % 3] / |c[a]|, both in [-1, 1];
  * s = st(u), t = st(v) with the linear transform st(w) = (1 + w) / 2
    (one of the projections S2 itself offers; the paper names none);
  * i = clamp(floor(2^30 s), 0, 2^30 - 1), j likewise from t;
  * Hilbert position d of (i, j) on the 2^30 x 2^30 grid, most significant
    level first: quadrant (rx, ry) -> digit (3 rx) xor ry, i.e. the first
    level visits (0,0), (0,1), (1,1), (1,0); inside quadrants with ry = 0 the
    sub-square is reflected (when rx = 1) and transposed;
  * id = face << 61 | d << 1 | 1 (a level-30 leaf).

Everything here follows these definitions directly, one level at a time.
"""
from __future__ import annotations

import numpy as np

MAX_LEVEL = 30
N = 1 << MAX_LEVEL


def st_from_uv(w):
    return 0.5 * (1.0 + np.asarray(w, dtype=np.float64))


def uv_from_st(s):
    return 2.0 * np.asarray(s, dtype=np.float64) - 1.0


def xyz(lat, lng):
    phi = np.radians(np.asarray(lat, dtype=np.float64))
    lam = np.radians(np.asarray(lng, dtype=np.float64))
    return np.cos(phi) * np.cos(lam), np.cos(phi) * np.sin(lam), np.sin(phi)


def project(lat, lng):
    """(lat, lng) degrees -> (face, u, v, s, t) as 1-D arrays (fp64, face int64)."""
    x, y, z = xyz(np.atleast_1d(lat), np.atleast_1d(lng))
    c = np.stack([x, y, z])
    ac = np.abs(c)
    a = np.where((ac[0] >= ac[1]) & (ac[0] >= ac[2]), 0, np.where(ac[1] >= ac[2], 1, 2))
    idx = np.arange(c.shape[1])
    major = c[a, idx]
    face = a + 3 * (major < 0)
    u = c[(a + 1) % 3, idx] / np.abs(major)
    v = c[(a + 2) % 3, idx] / np.abs(major)
    return face.astype(np.int64), u, v, st_from_uv(u), st_from_uv(v)


def leaf_ij(s, t):
    i = np.clip(np.floor(s * N), 0, N - 1).astype(np.int64)
    j = np.clip(np.floor(t * N), 0, N - 1).astype(np.int64)
    return i, j


def hilbert_d(i, j, levels: int = MAX_LEVEL):
    """Hilbert position of (i, j) on a 2^levels grid (vectorised)."""
    x = np.asarray(i, dtype=np.int64).copy()
    y = np.asarray(j, dtype=np.int64).copy()
    d = np.zeros_like(x)
    for b in range(levels - 1, -1, -1):
        rx = (x >> b) & 1
        ry = (y >> b) & 1
        d = (d << 2) | ((3 * rx) ^ ry)
        low = (1 << b) - 1
        x &= low
        y &= low
        flip = (ry == 0) & (rx == 1)
        x = np.where(flip, low - x, x)
        y = np.where(flip, low - y, y)
        swap = ry == 0
        x, y = np.where(swap, y, x), np.where(swap, x, y)
    return d


def hilbert_ij(d, levels: int = MAX_LEVEL):
    """Inverse of hilbert_d: rebuild (i, j) from the least significant level
    upwards, undoing each level's transform."""
    d = np.asarray(d, dtype=np.int64)
    x = np.zeros_like(d)
    y = np.zeros_like(d)
    for b in range(levels):
        digit = (d >> (2 * b)) & 3
        rx = (digit >> 1) & 1
        ry = (digit & 1) ^ rx
        low = (1 << b) - 1
        swap = ry == 0
        x, y = np.where(swap, y, x), np.where(swap, x, y)
        flip = (ry == 0) & (rx == 1)
        x = np.where(flip, low - x, x)
        y = np.where(flip, low - y, y)
        x = x | (rx << b)
        y = y | (ry << b)
    return x, y


def cell_ids(lat, lng) -> np.ndarray:
    """Level-30 cell ids (uint64) of fp64 (lat, lng) degree arrays."""
    face, _, _, s, t = project(lat, lng)
    i, j = leaf_ij(s, t)
    d = hilbert_d(i, j).astype(np.uint64)
    return (face.astype(np.uint64) << np.uint64(61)) | (d << np.uint64(1)) | np.uint64(1)


def decode_leaf(ids):
    """Leaf id -> (face, i, j)."""
    ids = np.asarray(ids, dtype=np.uint64)
    face = (ids >> np.uint64(61)).astype(np.int64)
    d = ((ids >> np.uint64(1)) & np.uint64((1 << 60) - 1)).astype(np.int64)
    i, j = hilbert_ij(d)
    return face, i, j


def parent(ids, level: int):
    """Ancestor at `level` of leaf ids: keep face + 2*level bits, set the
    marker bit right below them."""
    ids = np.asarray(ids, dtype=np.uint64)
    lsb = np.uint64(1) << np.uint64(2 * (MAX_LEVEL - level))
    return (ids & ~(lsb * np.uint64(2) - np.uint64(1))) | lsb


def is_valid_point(lat, lng):
    lat = np.asarray(lat, dtype=np.float64)
    lng = np.asarray(lng, dtype=np.float64)
    return np.isfinite(lat) & np.isfinite(lng) & (np.abs(lat) <= 90) & (np.abs(lng) <= 180)
