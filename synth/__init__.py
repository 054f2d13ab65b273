"""Seeded synthetic inputs for the point/polygon join.

This module only *draws* inputs: polygon partitions and point streams with the
shapes, sizes and distributions of the paper's workloads (Section "Evaluation":
NYC boroughs / neighbourhoods / census blocks joined with 1.23 B taxi points).
Those data sets are not available, so seeded stand-ins are generated here.
It contains none of the join's arithmetic (no cell ids, no point-in-polygon
test, no index): both the oracle and the GPU library consume what it returns.

Coordinates are fp64 degrees, stored as (lat, lng) pairs.

Polygon container (CSR, the layout the C ABI takes):
    verts          (V, 2) float64, (lat, lng) per vertex
    ring_off       (R + 1,) int64, ring r spans verts[ring_off[r]:ring_off[r+1]]
    poly_ring_off  (P + 1,) int32, polygon p owns rings poly_ring_off[p]..[p+1]
Ring 0 of a polygon is its outer ring, further rings are holes. Rings close
implicitly (the last vertex connects back to the first); orientation is
arbitrary.

Point streams are generated in fixed chunks of 2**20 points, chunk c drawing
from PCG64(SeedSequence([seed, c])), so any sub-range of a stream (a batch,
a sample) can be produced without generating what precedes it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# Bounding box of the synthetic city: lat [40.49, 40.92], lng [-74.27, -73.68].
BOX = (40.49, 40.92, -74.27, -73.68)
EARTH_R_M = 6371008.8
M_PER_DEG = EARTH_R_M * math.pi / 180.0  # metres per degree of arc
CHUNK = 1 << 20


def _rng(*key: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence(list(key))))


@dataclass
class Polygons:
    verts: np.ndarray
    ring_off: np.ndarray
    poly_ring_off: np.ndarray

    @property
    def n_polys(self) -> int:
        return int(self.poly_ring_off.shape[0] - 1)

    @property
    def n_verts(self) -> int:
        return int(self.verts.shape[0])

    def rings(self, p: int) -> list[np.ndarray]:
        r0, r1 = int(self.poly_ring_off[p]), int(self.poly_ring_off[p + 1])
        return [self.verts[self.ring_off[r]:self.ring_off[r + 1]] for r in range(r0, r1)]

    @classmethod
    def from_rings(cls, polys: list[list]) -> "Polygons":
        """polys[p] = [outer, hole, ...], each an (k, 2) array-like of (lat, lng)."""
        verts, ring_off, poly_ring_off = [], [0], [0]
        for rings in polys:
            for ring in rings:
                a = np.asarray(ring, dtype=np.float64).reshape(-1, 2)
                verts.append(a)
                ring_off.append(ring_off[-1] + a.shape[0])
            poly_ring_off.append(len(ring_off) - 1)
        v = np.concatenate(verts) if verts else np.zeros((0, 2))
        return cls(np.ascontiguousarray(v, dtype=np.float64),
                   np.asarray(ring_off, dtype=np.int64),
                   np.asarray(poly_ring_off, dtype=np.int32))

    def subset(self, ids) -> "Polygons":
        return Polygons.from_rings([self.rings(int(p)) for p in ids])


# --------------------------------------------------------------------------
# Gaussian mixture (shared by point streams and the fine partition's sites)
# --------------------------------------------------------------------------

@dataclass
class Mixture:
    """64 isotropic Gaussians in metres; centres uniform in the box,
    sigma log-uniform in [200 m, 2 km], equal weights."""
    centers: np.ndarray   # (K, 2) lat, lng
    sigma_m: np.ndarray   # (K,)

    @classmethod
    def make(cls, seed: int, k: int = 64, box=BOX) -> "Mixture":
        g = _rng(seed)
        lat = g.uniform(box[0], box[1], k)
        lng = g.uniform(box[2], box[3], k)
        sig = np.exp(g.uniform(math.log(200.0), math.log(2000.0), k))
        return cls(np.stack([lat, lng], 1), sig)

    def draw(self, g: np.random.Generator, n: int, sigma_scale: float = 1.0) -> np.ndarray:
        c = g.integers(0, self.centers.shape[0], n)
        z = g.standard_normal((n, 2))
        s_lat = self.sigma_m[c] * sigma_scale / M_PER_DEG
        s_lng = s_lat / np.cos(np.radians(self.centers[c, 0]))
        out = np.empty((n, 2))
        out[:, 0] = self.centers[c, 0] + z[:, 0] * s_lat
        out[:, 1] = self.centers[c, 1] + z[:, 1] * s_lng
        return out


def _uniform_box(g: np.random.Generator, n: int, box=BOX) -> np.ndarray:
    out = np.empty((n, 2))
    out[:, 0] = g.uniform(box[0], box[1], n)
    out[:, 1] = g.uniform(box[2], box[3], n)
    return out


def _fill_chunks(n_start: int, n_stop: int, seed: int, draw_chunk) -> np.ndarray:
    out = np.empty((max(0, n_stop - n_start), 2), dtype=np.float64)
    c0, c1 = n_start // CHUNK, (n_stop + CHUNK - 1) // CHUNK
    for c in range(c0, c1):
        lo, hi = c * CHUNK, (c + 1) * CHUNK
        chunk = draw_chunk(_rng(seed, c), CHUNK)
        a, b = max(lo, n_start), min(hi, n_stop)
        if a < b:
            out[a - n_start:b - n_start] = chunk[a - lo:b - lo]
    return out


def uniform_points(n_start: int, n_stop: int, seed: int, box=BOX) -> np.ndarray:
    """Points n_start..n_stop-1 of a uniform stream over the box."""
    return _fill_chunks(n_start, n_stop, seed, lambda g, m: _uniform_box(g, m, box))


def mixture_points(n_start: int, n_stop: int, seed: int, mixture: Mixture,
                   uniform_frac: float = 0.10, box=BOX) -> np.ndarray:
    """Points n_start..n_stop-1 of a stream: (1-uniform_frac) from the mixture,
    uniform_frac uniform in the box. Not clipped: mixture tails leave the box."""
    def draw(g, m):
        pts = mixture.draw(g, m)
        uni = g.random(m) < uniform_frac
        pts[uni] = _uniform_box(g, int(uni.sum()), box)
        return pts
    return _fill_chunks(n_start, n_stop, seed, draw)


# --------------------------------------------------------------------------
# Voronoi partitions with shared, jittered edges
# --------------------------------------------------------------------------

def _seg_cross(p, q, r, s, eps):
    """Vectorised closed segment intersection test pq vs rs (floats, with a
    tolerance that errs towards 'intersects'); used only to reject drawn
    polygons that are not simple."""
    def orient(a, b, c):
        return (b[..., 0] - a[..., 0]) * (c[..., 1] - a[..., 1]) - \
               (b[..., 1] - a[..., 1]) * (c[..., 0] - a[..., 0])
    d1, d2 = orient(p, q, r), orient(p, q, s)
    d3, d4 = orient(r, s, p), orient(r, s, q)
    t = math.sqrt(eps)
    box = ((np.minimum(p[..., 0], q[..., 0]) <= np.maximum(r[..., 0], s[..., 0]) + t) &
           (np.minimum(r[..., 0], s[..., 0]) <= np.maximum(p[..., 0], q[..., 0]) + t) &
           (np.minimum(p[..., 1], q[..., 1]) <= np.maximum(r[..., 1], s[..., 1]) + t) &
           (np.minimum(r[..., 1], s[..., 1]) <= np.maximum(p[..., 1], q[..., 1]) + t))
    return ((d1 * d2) <= eps) & ((d3 * d4) <= eps) & box


def _ring_simple(ring: np.ndarray) -> bool:
    m = ring.shape[0]
    if m < 3:
        return False
    a, b = ring, np.roll(ring, -1, axis=0)
    scale = float(np.abs(ring).max()) + 1.0
    eps = (1e-14 * scale) ** 2
    i, j = np.triu_indices(m, k=2)
    keep = ~((i == 0) & (j == m - 1))
    i, j = i[keep], j[keep]
    if i.size == 0:
        return True
    hit = _seg_cross(a[i], b[i], a[j], b[j], eps)
    return not bool(hit.any())


def _rings_disjoint(r1: np.ndarray, r2: np.ndarray) -> bool:
    a1, b1 = r1, np.roll(r1, -1, axis=0)
    a2, b2 = r2, np.roll(r2, -1, axis=0)
    i, j = np.meshgrid(np.arange(len(r1)), np.arange(len(r2)), indexing="ij")
    i, j = i.ravel(), j.ravel()
    scale = float(max(np.abs(r1).max(), np.abs(r2).max())) + 1.0
    return not bool(_seg_cross(a1[i], b1[i], a2[j], b2[j], (1e-14 * scale) ** 2).any())


def _point_seg_dist(p, a, b):
    ab = b - a
    t = np.clip(((p - a) * ab).sum(-1) / np.maximum((ab * ab).sum(-1), 1e-300), 0.0, 1.0)
    d = a + t[:, None] * ab - p
    return np.sqrt((d * d).sum(-1))


def voronoi_partition(n: int, seed: int, *, seg_per_edge=10.0, vert_target=None,
                      hole_frac: float = 0.0, jitter: float = 0.2,
                      site_mixture: Mixture | None = None, site_mix_frac: float = 0.0,
                      site_sigma_scale: float = 1.0, box=BOX) -> Polygons:
    """Seeded Voronoi partition of the box into n polygons.

    * Sites live in a local metric frame (x scaled by cos of the box's mid
      latitude); cells are clipped to the box by mirroring the sites across
      its four sides.
    * Every Voronoi edge is subdivided; interior edges get a perpendicular
      jitter drawn from a generator keyed by (seed, site pair), and both
      neighbours use the identical fp64 polyline, so the partition has no
      gaps or overlaps. Box-side edges are subdivided, not jittered.
    * Segments per edge: `seg_per_edge`, or, when `vert_target=(lo, hi)`, a
      per-polygon vertex target drawn log-uniform in [lo, hi] spread over the
      polygon's edges (a shared edge uses the mean of its two neighbours).
    * `hole_frac` of the polygons receive one hole: a jittered 12..24-gon
      around the site at 0.3x the site's distance to its outer ring. The hole
      region belongs to no polygon.
    * Polygons that come out non-simple get their edges' jitter halved and
      are redrawn (at most 6 times, then jitter 0: straight subdivided edges
      of a convex cell are simple).
    """
    from scipy.spatial import Voronoi

    g = _rng(seed)
    lat0 = 0.5 * (box[0] + box[1])
    kx = math.cos(math.radians(lat0))
    W, H = (box[3] - box[2]) * kx, box[1] - box[0]

    # sites in the local frame
    sites = np.empty((0, 2))
    while sites.shape[0] < n:
        need = n - sites.shape[0]
        if site_mixture is not None and site_mix_frac > 0:
            nm = int(round(need * site_mix_frac))
            mpts = site_mixture.draw(g, nm, site_sigma_scale)
            upts = _uniform_box(g, need - nm, box)
            cand = np.concatenate([mpts, upts])
        else:
            cand = _uniform_box(g, need, box)
        fx = (cand[:, 1] - box[2]) * kx
        fy = cand[:, 0] - box[0]
        ok = (fx > 0) & (fx < W) & (fy > 0) & (fy < H)
        sites = np.concatenate([sites, np.stack([fx[ok], fy[ok]], 1)])
    sites = sites[:n]
    # drop exact duplicates (vanishingly unlikely) by a tiny deterministic nudge
    mir = np.concatenate([sites,
                          np.stack([-sites[:, 0], sites[:, 1]], 1),
                          np.stack([2 * W - sites[:, 0], sites[:, 1]], 1),
                          np.stack([sites[:, 0], -sites[:, 1]], 1),
                          np.stack([sites[:, 0], 2 * H - sites[:, 1]], 1)])
    vor = Voronoi(mir)
    V = vor.vertices.copy()
    tol = 1e-9 * max(W, H)
    V[np.abs(V[:, 0]) < tol, 0] = 0.0
    V[np.abs(V[:, 0] - W) < tol, 0] = W
    V[np.abs(V[:, 1]) < tol, 1] = 0.0
    V[np.abs(V[:, 1] - H) < tol, 1] = H

    # per-polygon per-edge segment targets
    regions = [vor.regions[vor.point_region[k]] for k in range(n)]
    if vert_target is not None:
        lo, hi = vert_target
        tgt = np.exp(g.uniform(math.log(lo), math.log(hi), n))
        per_edge = np.array([tgt[k] / max(3, len(regions[k])) for k in range(n)])
    else:
        per_edge = np.full(n, float(seg_per_edge))
    hole_draw = g.random(n) < hole_frac
    hole_seeds = g.integers(0, 2**31 - 1, n)

    # ridge lookup: unordered vertex pair -> (site p, site q)
    ridge_of = {}
    for (p, q), (va, vb) in zip(vor.ridge_points, vor.ridge_vertices):
        if p >= n and q >= n:
            continue
        if va < 0 or vb < 0:
            continue
        ridge_of[(min(va, vb), max(va, vb))] = (int(p), int(q))

    def to_latlng(xy):
        out = np.empty_like(xy)
        out[:, 0] = box[0] + xy[:, 1]
        out[:, 1] = box[2] + xy[:, 0] / kx
        return out

    V_ll = to_latlng(V)
    amp = {}  # ridge key -> jitter amplitude
    cache = {}

    def polyline(key):
        """Interior points (lat/lng) of the ridge polyline from key[0] to key[1]."""
        if key in cache:
            return cache[key]
        va, vb = key
        p, q = ridge_of[key]
        interior = p < n and q < n
        if interior:
            m = int(max(1, round(0.5 * (per_edge[p] + per_edge[q]))))
        else:
            m = int(max(1, round(per_edge[min(p, q)])))
        A, B = V[va], V[vb]
        if m <= 1:
            pts = np.zeros((0, 2))
        else:
            t = np.arange(1, m) / m
            pts = A + t[:, None] * (B - A)
            if interior:
                a = amp.get(key, jitter)
                d = B - A
                nrm = np.array([-d[1], d[0]]) / max(np.hypot(*d), 1e-300)
                gr = _rng(seed, 7, min(p, q), max(p, q))
                off = gr.uniform(-1.0, 1.0, m - 1) * a * (np.hypot(*d) / m)
                pts = pts + off[:, None] * nrm[None, :]
        res = to_latlng(pts) if pts.shape[0] else np.zeros((0, 2))
        cache[key] = res
        return res

    def outer_ring(k):
        reg = regions[k]
        parts = []
        for a_i in range(len(reg)):
            va, vb = reg[a_i], reg[(a_i + 1) % len(reg)]
            key = (min(va, vb), max(va, vb))
            parts.append(V_ll[va][None, :])
            pl = polyline(key)
            parts.append(pl if va == key[0] else pl[::-1])
        ring = np.concatenate(parts)
        # drop consecutive exact duplicates (e.g. snapped corners)
        keep = np.ones(len(ring), bool)
        keep[1:] = np.any(ring[1:] != ring[:-1], axis=1)
        if np.all(ring[-1] == ring[0]) and len(ring) > 1:
            keep[-1] = False
        return ring[keep]

    rings = [None] * n
    todo = list(range(n))
    for attempt in range(8):
        bad = []
        for k in todo:
            r = outer_ring(k)
            rings[k] = r
            if not _ring_simple(r):
                bad.append(k)
        if not bad:
            break
        todo = set()
        for k in bad:
            reg = regions[k]
            for a_i in range(len(reg)):
                va, vb = reg[a_i], reg[(a_i + 1) % len(reg)]
                key = (min(va, vb), max(va, vb))
                amp[key] = 0.0 if attempt >= 5 else amp.get(key, jitter) * 0.5
                cache.pop(key, None)
                p, q = ridge_of[key]
                todo.update(x for x in (p, q) if x < n)
        todo = sorted(todo)
    else:
        raise RuntimeError("voronoi_partition: could not draw simple polygons")

    polys = []
    for k in range(n):
        outer = rings[k]
        entry = [outer]
        if hole_draw[k]:
            site_ll = to_latlng(sites[k:k + 1])[0]
            a, b = outer, np.roll(outer, -1, axis=0)
            # distances in the local frame (degrees of latitude)
            sc = np.array([1.0, kx])
            d = _point_seg_dist(site_ll[None, :] * sc, a * sc, b * sc).min()
            hg = _rng(int(hole_seeds[k]))
            m = int(hg.integers(12, 25))
            ang = np.sort(hg.uniform(0, 2 * math.pi, m))
            rad = 0.3 * d * hg.uniform(0.8, 1.2, m)
            hole = np.stack([site_ll[0] + rad * np.sin(ang),
                             site_ll[1] + rad * np.cos(ang) / kx], 1)
            if _ring_simple(hole) and _rings_disjoint(hole, outer):
                entry.append(hole)
        polys.append(entry)
    return Polygons.from_rings(polys)


# --------------------------------------------------------------------------
# The workloads
# --------------------------------------------------------------------------

WORKLOADS = {
    # 16 Voronoi polygons, ~60 vertices each, 1e5 uniform points, exact mode,
    # covering cells up to level 20.
    "c1": dict(n_polys=16, poly_seed=1001, seg_per_edge=10.0, vert_target=None,
               hole_frac=0.0, n_points=100_000, point_seed=2001, points="uniform",
               mixture_seed=3001),
    # 290 polygons, vertex counts log-uniform 20..800, 5% with one hole;
    # 1e8 points: 64-component Gaussian mixture + 10% uniform.
    "c2": dict(n_polys=290, poly_seed=1002, seg_per_edge=None, vert_target=(20, 800),
               hole_frac=0.05, n_points=100_000_000, point_seed=2002, points="mixture",
               mixture_seed=3002),
    # 40,000 small polygons (~20 vertices), sites 70% from the mixture with
    # doubled sigma + 30% uniform; 1e9 points streamed in 2**24-point batches.
    "c3": dict(n_polys=40_000, poly_seed=1003, seg_per_edge=3.3, vert_target=None,
               hole_frac=0.0, n_points=1_000_000_000, point_seed=2003, points="mixture",
               mixture_seed=3002, site_mix_frac=0.7, site_sigma_scale=2.0,
               batch=1 << 24),
}


def workload_polygons(name: str) -> Polygons:
    w = WORKLOADS[name]
    mix = Mixture.make(w["mixture_seed"]) if w.get("site_mix_frac") else None
    return voronoi_partition(
        w["n_polys"], w["poly_seed"], seg_per_edge=w["seg_per_edge"] or 10.0,
        vert_target=w["vert_target"], hole_frac=w["hole_frac"],
        site_mixture=mix, site_mix_frac=w.get("site_mix_frac", 0.0),
        site_sigma_scale=w.get("site_sigma_scale", 1.0))


def workload_points(name: str, start: int = 0, stop: int | None = None) -> np.ndarray:
    w = WORKLOADS[name]
    stop = w["n_points"] if stop is None else stop
    if w["points"] == "uniform":
        return uniform_points(start, stop, w["point_seed"])
    return mixture_points(start, stop, w["point_seed"], Mixture.make(w["mixture_seed"]))


def training_points(name: str, n: int) -> np.ndarray:
    """Historical points for training a workload's index: the workload's own
    point distribution, drawn from a different seed (point seed + 5000)."""
    w = WORKLOADS[name]
    seed = w["point_seed"] + 5000
    if w["points"] == "uniform":
        return uniform_points(0, n, seed)
    return mixture_points(0, n, seed, Mixture.make(w["mixture_seed"]))


def batch_sizes(n_batches: int, seed: int, hi: float = 1e6) -> np.ndarray:
    """Uneven batch sizes floor(exp(U(0, ln hi))), at least 1."""
    g = _rng(seed)
    return np.maximum(1, np.floor(np.exp(g.uniform(0.0, math.log(hi), n_batches)))).astype(np.int64)
