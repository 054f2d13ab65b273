"""Pins for the oracle (CPU): the brute-force join is checked against what the
paper and plain mathematics fix, never against itself.

* exact orientation sign vs rational arithmetic (fractions.Fraction);
* hand-built polygons with hand-derived answers under the ST_Covers rule
  (Section "Background": points on edges and vertices are inside);
* convex polygons: crossing number == intersection of closed half-planes;
* Monte Carlo hit fraction vs shoelace area;
* a Voronoi partition covers each generic point exactly once;
* invariance under ring reversal / rotation / exact dyadic translation;
* the bounding-box prefilter changes nothing.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth


def frac_orient(a, b, p):
    ax, ay, bx, by, px, py = (Fraction(float(v)) for v in (*a, *b, *p))
    d = (bx - ax) * (py - ay) - (by - ay) * (px - ax)
    return (d > 0) - (d < 0)


def int_orient(a, b, p):
    """Exact sign by integer arithmetic: every finite double is an integer
    multiple of 2^-1074, so scaling all six coordinates by 2^1074 turns the
    determinant into an exact integer expression."""
    def sc(v):
        num, den = float(v).as_integer_ratio()
        return num << (1075 - den.bit_length())
    ax, ay, bx, by, px, py = (sc(v) for v in (*a, *b, *p))
    d = (bx - ax) * (py - ay) - (by - ay) * (px - ax)
    return (d > 0) - (d < 0)


def adversarial_triples(rng, n):
    """(n, 6) rows (ax, ay, bx, by, px, py) of five kinds: generic; near the
    line through a and b (rounded, nudged by ulps); exactly collinear dyadic;
    lat/lng-like with tiny offsets from an edge; widely different
    magnitudes."""
    kind = rng.integers(0, 5, n)
    out = np.empty((n, 6))
    k = kind == 0
    out[k] = rng.uniform(-180, 180, (k.sum(), 6))
    k = kind == 1
    m = k.sum()
    a, b = rng.uniform(-75, -73, (m, 2)), rng.uniform(-75, -73, (m, 2))
    p = a + rng.uniform(-0.5, 1.5, (m, 1)) * (b - a)
    p = p + rng.integers(-3, 4, (m, 2)) * np.spacing(p)
    out[k] = np.concatenate([a, b, p], 1)
    k = kind == 2
    m = k.sum()
    a = rng.integers(-2**20, 2**20, (m, 2)) / 2.0**10
    d = rng.integers(-2**10, 2**10, (m, 2)) / 2.0**12
    out[k] = np.concatenate([a, a + d, a + rng.integers(-4, 5, (m, 1)) * d], 1)
    k = kind == 3
    m = k.sum()
    a = np.stack([rng.uniform(-74.3, -73.6, m), rng.uniform(40.4, 41.0, m)], 1)
    b = a + rng.uniform(-1e-3, 1e-3, (m, 2))
    p = a + rng.uniform(0, 1, (m, 1)) * (b - a) + rng.uniform(-1e-15, 1e-15, (m, 2))
    out[k] = np.concatenate([a, b, p], 1)
    k = kind == 4
    m = k.sum()
    a = rng.uniform(-1, 1, (m, 2)) * 10.0 ** rng.integers(-30, 3, (m, 2))
    b = rng.uniform(-1, 1, (m, 2)) * 10.0 ** rng.integers(-30, 3, (m, 2))
    out[k] = np.concatenate([a, b, a + rng.uniform(0, 1, (m, 1)) * (b - a)], 1)
    return out


def test_orient_sign_matches_rationals():
    """1e6 adversarial triples: the oracle's filtered and exact-only signs
    equal the sign of the exact integer determinant (and, on the first
    20,000, of the same determinant in fractions.Fraction)."""
    rng = np.random.default_rng(11)
    rows = adversarial_triples(rng, 1_000_000)
    want = np.array([int_orient(r[0:2], r[2:4], r[4:6]) for r in rows], dtype=np.int8)
    for r, w in zip(rows[:20000], want[:20000]):
        assert frac_orient(r[0:2], r[2:4], r[4:6]) == w
    got = oracle.orient_signs(rows)
    got_exact = oracle.orient_signs(rows, exact_only=True)
    bad = np.nonzero((got != want) | (got_exact != want))[0]
    assert bad.size == 0, rows[bad[:3]]
    assert (want == 0).sum() > 20000  # the adversarial set really exercises the exact path
    # the single-call entry agrees with the batched one
    for r, w in zip(rows[:2000], want[:2000]):
        assert oracle.orient_sign(r[0:2], r[2:4], r[4:6]) == w


def _P(*rings_xy):
    """Polygon from rings given as (x=lng, y=lat) pairs."""
    return [np.asarray(r, dtype=np.float64)[:, ::-1] for r in rings_xy]


def _covers(poly_rings, x, y):
    P = synth.Polygons.from_rings([poly_rings])
    return oracle.covers(P, 0, lat=y, lng=x)


SQUARE = _P([(0, 0), (0, 1), (1, 1), (1, 0)])
U_SHAPE = _P([(0, 0), (3, 0), (3, 3), (2, 3), (2, 1), (1, 1), (1, 3), (0, 3)])
HOLED = _P([(0, 0), (4, 0), (4, 4), (0, 4)], [(1, 1), (3, 1), (3, 3), (1, 3)])
DIAMOND = _P([(0, 1), (1, 0), (2, 1), (1, 2)])
TRIANGLE = _P([(0, 0), (4, 0), (2, 2)])

E = 2.0 ** -40

HAND = [
    # unit square
    (SQUARE, 0.5, 0.5, True), (SQUARE, 1.5, 0.5, False), (SQUARE, 0.5, 0.0, True),
    (SQUARE, 0.0, 0.0, True), (SQUARE, 1.0, 1.0, True), (SQUARE, 0.5, -E, False),
    (SQUARE, 0.5, E, True), (SQUARE, 1.0 + E, 0.5, False), (SQUARE, 1.0, 0.5, True),
    (SQUARE, -E, -E, False),
    # U shape (concave): notch between the arms is outside
    (U_SHAPE, 1.5, 2.0, False), (U_SHAPE, 0.5, 2.0, True), (U_SHAPE, 2.5, 2.0, True),
    (U_SHAPE, 1.5, 0.5, True), (U_SHAPE, 0.5, 1.0, True), (U_SHAPE, 1.5, 1.0, True),
    (U_SHAPE, 2.5, 1.0, True), (U_SHAPE, 3.5, 1.0, False), (U_SHAPE, -0.5, 1.0, False),
    (U_SHAPE, 1.5, 3.0, False), (U_SHAPE, 1.0, 3.0, True), (U_SHAPE, 1.5, 1.0 + E, False),
    # square with a square hole: hole boundary is boundary (covered)
    (HOLED, 0.5, 0.5, True), (HOLED, 2.0, 2.0, False), (HOLED, 1.0, 2.0, True),
    (HOLED, 1.0, 1.0, True), (HOLED, 3.5, 2.0, True), (HOLED, 1.0 + E, 2.0, False),
    (HOLED, 1.0 - E, 2.0, True), (HOLED, 2.0, 3.0, True), (HOLED, 4.0, 4.0, True),
    # diamond: horizontal rays through vertices
    (DIAMOND, 0.5, 1.0, True), (DIAMOND, -0.5, 1.0, False), (DIAMOND, 3.0, 1.0, False),
    (DIAMOND, 1.0, 0.0, True), (DIAMOND, 1.0, -E, False), (DIAMOND, 2.0, 1.0, True),
    (DIAMOND, 1.5, 1.5, True), (DIAMOND, 1.5 + E, 1.5, False),
    # triangle with a horizontal edge at the point's latitude
    (TRIANGLE, -1.0, 0.0, False), (TRIANGLE, 5.0, 0.0, False), (TRIANGLE, 2.0, 0.0, True),
    (TRIANGLE, 2.0, 1.0, True), (TRIANGLE, 2.0, 2.0, True), (TRIANGLE, 2.0, 2.0 + E, False),
    (TRIANGLE, 1.0, 1.0, True), (TRIANGLE, 1.0 - E, 1.0, False),
]


@pytest.mark.parametrize("rings,x,y,want", HAND)
def test_hand_built_polygons(rings, x, y, want):
    assert _covers(rings, x, y) == want
    # ring orientation and start vertex do not matter
    rev = [r[::-1] for r in rings]
    assert _covers(rev, x, y) == want
    rot = [np.roll(r, 1, axis=0) for r in rings]
    assert _covers(rot, x, y) == want


def _convex_hull(pts):
    pts = sorted(map(tuple, pts))

    def cross(o, a, b):
        return (Fraction(a[0]) - Fraction(o[0])) * (Fraction(b[1]) - Fraction(o[1])) - \
               (Fraction(a[1]) - Fraction(o[1])) * (Fraction(b[0]) - Fraction(o[0]))
    lower, upper = [], []
    for p in pts:
        while len(lower) >= 2 and cross(lower[-2], lower[-1], p) <= 0:
            lower.pop()
        lower.append(p)
    for p in reversed(pts):
        while len(upper) >= 2 and cross(upper[-2], upper[-1], p) <= 0:
            upper.pop()
        upper.append(p)
    return lower[:-1] + upper[:-1]  # counter-clockwise


def test_convex_equals_halfplane_intersection():
    """For a convex polygon, covered <=> on the inner closed side of every edge."""
    rng = np.random.default_rng(5)
    checked = 0
    for trial in range(40):
        c = rng.uniform([-74.2, 40.5], [-73.7, 40.9])
        hull = _convex_hull(c + rng.normal(0, 0.01, (12, 2)))
        rings = [np.asarray(hull)[:, ::-1]]
        P = synth.Polygons.from_rings([rings])
        lo, hi = np.min(hull, 0), np.max(hull, 0)
        pts = list(rng.uniform(lo - 0.002, hi + 0.002, (150, 2)))
        # boundary points: vertices and exact dyadic midpoints of axis-aligned-ish edges
        pts += [np.array(v) for v in hull[:4]]
        for (x, y) in pts:
            want = all(frac_orient(hull[k], hull[(k + 1) % len(hull)], (x, y)) >= 0
                       for k in range(len(hull)))
            assert oracle.covers(P, 0, lat=y, lng=x) == want
            checked += 1
    assert checked > 5000


def test_monte_carlo_area_matches_shoelace():
    P = synth.workload_polygons("c2")
    rng = np.random.default_rng(7)
    for p in [0, 17, 101, 250]:
        rings = P.rings(p)
        area = 0.0
        for r in rings:
            x, y = r[:, 1], r[:, 0]
            area_r = 0.5 * abs(np.dot(x, np.roll(y, -1)) - np.dot(y, np.roll(x, -1)))
            area += area_r if area == 0.0 else -area_r  # holes subtract
        lo, hi = rings[0].min(0), rings[0].max(0)
        box_area = (hi[0] - lo[0]) * (hi[1] - lo[1])
        n = 40000
        pts = rng.uniform(lo, hi, (n, 2))
        sub = P.subset([p])
        res = oracle.join(sub, pts)
        frac = float((res.out == 0).mean())
        expect = area / box_area
        sigma = np.sqrt(expect * (1 - expect) / n)
        assert abs(frac - expect) < 5 * sigma + 1e-12, (p, frac, expect)


def test_partition_covers_generic_points_once():
    P = synth.workload_polygons("c1")
    pts = synth.uniform_points(0, 200000, seed=77)
    res = oracle.join(P, pts)
    # generic points: exactly one polygon each
    assert np.all(res.cnt == 1)
    assert np.all(res.out >= 0)


def test_partition_shared_vertices_covered_by_all_neighbours():
    P = synth.workload_polygons("c1")
    v = P.verts
    # count, for each distinct vertex, how many polygons list it
    owners = {}
    for p in range(P.n_polys):
        for r in P.rings(p):
            for q in map(tuple, r):
                owners.setdefault(q, set()).add(p)
    keys = list(owners)
    pts = np.asarray(keys)
    res = oracle.join(P, pts)
    got = {}
    for i, o in enumerate(res.out):
        if o >= 0:
            got.setdefault(i, set()).add(int(o))
    for i, p in res.pairs:
        got.setdefault(int(i), set()).add(int(p))
    for i, k in enumerate(keys):
        # every polygon that has this vertex covers it (possibly more: a
        # vertex can also lie on another polygon's straight edge)
        assert owners[k] <= got.get(i, set()), (k, owners[k], got.get(i))
    assert v.shape[0] > 0


def test_dyadic_translation_invariance():
    P = synth.workload_polygons("c1")
    pts = synth.uniform_points(0, 20000, seed=78)
    base = oracle.join(P, pts)
    # +0.25 deg lat / +0.125 deg lng keeps every value in its binade: exact
    sh = np.array([0.25, 0.125])
    P2 = synth.Polygons(P.verts + sh, P.ring_off, P.poly_ring_off)
    assert np.array_equal(P2.verts - sh, P.verts)
    moved = oracle.join(P2, pts + sh)
    assert np.array_equal(base.out, moved.out)
    assert np.array_equal(base.pairs, moved.pairs)


def test_bbox_prefilter_changes_nothing():
    P = synth.workload_polygons("c1")
    pts = np.concatenate([synth.uniform_points(0, 5000, seed=79), P.verts[::3]])
    a = oracle.join(P, pts, use_bbox=True)
    b = oracle.join(P, pts, use_bbox=False)
    assert np.array_equal(a.out, b.out) and np.array_equal(a.pairs, b.pairs)


def test_out_of_domain_points_match_nothing():
    P = synth.Polygons.from_rings([[np.array([[-90, -180], [-90, 180], [90, 180], [90, -180]],
                                             dtype=float)]])
    pts = np.array([[np.nan, 0], [0, np.inf], [91, 0], [0, 181], [0, -180.0], [90, 0], [0, 0]])
    res = oracle.join(P, pts)
    assert res.out.tolist() == [-1, -1, -1, -1, 0, 0, 0]


def test_boundary_distance_checker():
    # 1 degree of latitude is R*pi/180 metres
    sq = synth.Polygons.from_rings([[np.array([[0, 0], [0, 1], [1, 1], [1, 0]], float)]])
    d = oracle.boundary_dist_m(sq, 0, lat=-1.0, lng=0.5)
    assert abs(d - synth.M_PER_DEG) < 1e-6
    d = oracle.boundary_dist_m(sq, 0, lat=0.5, lng=0.5)
    assert abs(d - 0.5 * synth.M_PER_DEG * np.cos(np.radians(0.5))) < 1e-6


# ---------------------------------------------------------- spherical model

def _gc_lat(lat_a, lng_a, lat_b, lng_b, lng):
    """Latitude of the great circle through a and b at longitude lng (closed
    form: tan(lat) is a combination of the endpoints' tangents weighted by
    the sines of the longitude differences)."""
    r = np.radians
    t = (np.tan(r(lat_a)) * np.sin(r(lng_b - lng)) + np.tan(r(lat_b)) * np.sin(r(lng - lng_a))) \
        / np.sin(r(lng_b - lng_a))
    return np.degrees(np.arctan(t))


def test_sphere_edges_bulge_poleward_by_the_closed_form():
    """A lat/lng rectangle whose east-west edges are great-circle arcs: at the
    middle longitude the southern edge lies north of its chord and the
    northern edge north of its own, by the closed form of the great circle's
    latitude. Points just inside and outside of each arc, and between arc
    and chord (where the planar and spherical models differ)."""
    sq = [np.array([[40.0, -75.0], [40.0, -73.0], [41.0, -73.0], [41.0, -75.0]])]
    P = synth.Polygons.from_rings([sq])
    south = _gc_lat(40.0, -75.0, 40.0, -73.0, -74.0)
    north = _gc_lat(41.0, -75.0, 41.0, -73.0, -74.0)
    assert south > 40.004 and north > 41.004
    eps = 1e-6
    for lat, want_sphere, want_plane in ((south + eps, True, True), (south - eps, False, True),
                                         ((40.0 + south) / 2, False, True),
                                         (north - eps, True, False), (north + eps, False, False),
                                         ((41.0 + north) / 2, True, False), (40.5, True, True),
                                         (39.99, False, False)):
        assert oracle.covers_sphere(P, 0, lat, -74.0) == want_sphere, lat
        assert oracle.covers(P, 0, lat, -74.0) == want_plane, lat
    # off the middle longitude the closed form still decides
    for lng in (-74.9, -74.3, -73.2):
        g = _gc_lat(40.0, -75.0, 40.0, -73.0, lng)
        assert oracle.covers_sphere(P, 0, g + eps, lng) and not oracle.covers_sphere(P, 0, g - eps, lng)


def test_sphere_vertices_meridians_and_reversal():
    """Vertices and points on a meridian edge are covered; reversing a ring
    or rotating its start changes nothing; far from edges the spherical and
    planar models agree (the arcs and chords differ by centimetres here)."""
    ring = np.array([[40.6, -74.1], [40.6, -73.9], [40.8, -73.9], [40.8, -74.0], [40.7, -74.1]])
    P = synth.Polygons.from_rings([[ring]])
    for lat, lng in ring:
        assert oracle.covers_sphere(P, 0, lat, lng)
    assert oracle.covers_sphere(P, 0, 40.7, -73.9)      # on the meridian edge
    assert not oracle.covers_sphere(P, 0, 40.7, -73.9 + 1e-9)
    rng = np.random.default_rng(12)
    pts = np.stack([rng.uniform(40.55, 40.85, 4000), rng.uniform(-74.15, -73.85, 4000)], 1)
    variants = [ring[::-1], np.roll(ring, 2, 0), np.roll(ring[::-1], 3, 0)]
    base = oracle.join_sphere(P, pts).out
    for v in variants:
        assert np.array_equal(oracle.join_sphere(synth.Polygons.from_rings([[v]]), pts).out, base)
    plane = oracle.join(P, pts).out
    far = oracle.boundary_dist_sphere_pairs(P, pts, np.stack([np.arange(len(pts)),
                                                              np.zeros(len(pts), np.int64)], 1)) > 1.0
    assert far.sum() > 3500 and np.array_equal(base[far], plane[far])


def test_sphere_partition_covers_generic_points_once():
    """The Voronoi partition's neighbours share identical arcs, so in the
    spherical model too every in-box point away from edges is covered by
    exactly one polygon (the holes of C2 excepted: C1 has none)."""
    P = synth.workload_polygons("c1")
    pts = synth.workload_points("c1", 0, 20000)
    res = oracle.join_sphere(P, pts)
    pairs = np.stack([np.arange(len(pts)), np.maximum(res.out, 0).astype(np.int64)], 1)
    far = oracle.boundary_dist_sphere_pairs(P, pts, pairs) > 0.01
    assert far.sum() > 19000
    assert np.all(res.cnt[far] == 1)
