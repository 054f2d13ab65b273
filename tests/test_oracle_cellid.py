"""Pins for the reference cell ids (CPU).

Section "Background" fixes the id layout (3 face bits, 2 bits per level, a
marker bit, zeros) and the one property the join relies on: a child's id
extends its parent's prefix. The Hilbert curve is pinned by its defining
properties (bijection, unit steps, self-similar prefix), the projection by
closed-form points and by inverting it.
"""
import numpy as np

from oracle import cellid as C


def test_hilbert_first_level_order():
    d = C.hilbert_d(np.array([0, 0, 1, 1]), np.array([0, 1, 1, 0]), 1)
    assert d.tolist() == [0, 1, 2, 3]


def test_hilbert_bijection_unit_steps_and_prefix():
    for L in range(1, 7):
        n = 1 << L
        i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        i, j = i.ravel(), j.ravel()
        d = C.hilbert_d(i, j, L)
        assert np.array_equal(np.sort(d), np.arange(n * n))
        order = np.argsort(d)
        step = np.abs(np.diff(i[order])) + np.abs(np.diff(j[order]))
        assert np.all(step == 1)
        if L > 1:
            # the parent cell's position is the child's position without its last digit
            assert np.array_equal(C.hilbert_d(i >> 1, j >> 1, L - 1), d >> 2)


def test_hilbert_roundtrip_level30():
    rng = np.random.default_rng(1)
    i = rng.integers(0, 1 << 30, 200000)
    j = rng.integers(0, 1 << 30, 200000)
    x, y = C.hilbert_ij(C.hilbert_d(i, j))
    assert np.array_equal(x, i) and np.array_equal(y, j)
    # consecutive level-30 positions are unit steps as well
    d = rng.integers(0, (1 << 60) - 1, 50000)
    a = np.stack(C.hilbert_ij(d))
    b = np.stack(C.hilbert_ij(d + 1))
    assert np.all(np.abs(a - b).sum(0) == 1)


def test_st_transform():
    assert C.st_from_uv(np.array([-1.0, 0.0, 1.0])).tolist() == [0.0, 0.5, 1.0]
    # the linear reading s = (1 + u) / 2 at interior points (a quadratic or
    # tangent transform gives 0.79 / 0.85 at u = 1/2)
    assert C.st_from_uv(np.array([-0.5, 0.5, 0.25])).tolist() == [0.25, 0.75, 0.625]
    w = np.linspace(-1, 1, 10001)
    s = C.st_from_uv(w)
    assert np.all(np.diff(s) > 0)
    assert np.allclose(C.uv_from_st(s), w, atol=1e-15, rtol=0)


def test_face_centres_and_numbering():
    lat = np.array([0, 0, 90, 0, 0, -90.0])
    lng = np.array([0, 90, 0, 180, -90, 0.0])
    face, u, v, s, t = C.project(lat, lng)
    assert face.tolist() == [0, 1, 2, 3, 4, 5]
    assert np.allclose(u, 0, atol=1e-15) and np.allclose(v, 0, atol=1e-15)
    # (0, 0): face 0, s = t = 1/2, i = j = 2^29: first digit 2, rest 0
    ids = C.cell_ids(np.array([0.0]), np.array([0.0]))
    assert int(ids[0]) == (2 << 59) | 1


def test_nyc_is_on_face_4():
    face, u, v, s, t = C.project(np.array([40.7]), np.array([-74.0]))
    assert face[0] == 4  # -y axis dominates at lng -74
    assert -1 <= u[0] <= 1 and -1 <= v[0] <= 1


def test_id_layout_and_parent_prefix():
    rng = np.random.default_rng(2)
    lat = rng.uniform(-90, 90, 100000)
    lng = rng.uniform(-180, 180, 100000)
    ids = C.cell_ids(lat, lng)
    assert np.all(ids & np.uint64(1) == 1)
    face = ids >> np.uint64(61)
    assert np.all(face <= 5)
    for L in (0, 1, 7, 20, 29, 30):
        par = C.parent(ids, L)
        lsb = np.uint64(1) << np.uint64(2 * (30 - L))
        # marker bit at 2 (30 - L), zeros below it
        assert np.all(par & (lsb * np.uint64(2) - np.uint64(1)) == lsb)
        # the parent is a bit prefix of the leaf
        sh = np.uint64(2 * (30 - L) + 1)
        assert np.all((par >> sh) == (ids >> sh))
        # descendants lie within [parent - lsb + 1, parent + lsb - 1]
        assert np.all(ids >= par - lsb + np.uint64(1)) and np.all(ids <= par + lsb - np.uint64(1))


def test_cell_centre_roundtrip():
    """Inverting the projection at a cell's centre lands in the same cell."""
    rng = np.random.default_rng(3)
    lat = rng.uniform(-89, 89, 50000)
    lng = rng.uniform(-179, 179, 50000)
    ids = C.cell_ids(lat, lng)
    face, i, j = C.decode_leaf(ids)
    s = (i + 0.5) / C.N
    t = (j + 0.5) / C.N
    u, v = C.uv_from_st(s), C.uv_from_st(t)
    a = face % 3
    sign = np.where(face >= 3, -1.0, 1.0)
    c = np.zeros((3, lat.size))
    idx = np.arange(lat.size)
    c[a, idx] = sign
    c[(a + 1) % 3, idx] = u
    c[(a + 2) % 3, idx] = v
    lat2 = np.degrees(np.arctan2(c[2], np.hypot(c[0], c[1])))
    lng2 = np.degrees(np.arctan2(c[1], c[0]))
    assert np.array_equal(C.cell_ids(lat2, lng2), ids)


def test_closed_form_leaf_off_centre():
    """A point off the face centre, derived by hand: on the equator at
    lng = atan(u) with u = 1/2 + 2^-30, the x axis dominates (face 0), u is
    y/x = tan(lng) and v = z/x = 0. The linear transform gives
    s = 3/4 + 2^-31, the middle of leaf column i = 3 * 2^28 (fp64 rounding
    moves s by about 1e-16, far from the column's edges), and t = 1/2, so
    j = 2^29 exactly. The Hilbert digits of that leaf follow from the curve's
    definition: level 1 has (i, j) bits (1, 1) -> digit 2; level 2 has bits
    (1, 0) -> digit 3, and that quadrant is reflected and transposed, which
    maps the remaining all-zero (i, j) bits to all ones -> digit 2 at every
    further level."""
    u = 0.5 + 2.0 ** -30
    lng = np.degrees(np.arctan(u))
    face, uu, vv, s, t = C.project(np.array([0.0]), np.array([lng]))
    assert face[0] == 0 and vv[0] == 0.0
    i, j = C.leaf_ij(s, t)
    assert (int(i[0]), int(j[0])) == (3 << 28, 1 << 29)
    d = 2
    d = (d << 2) | 3
    for _ in range(28):
        d = (d << 2) | 2
    ids = C.cell_ids(np.array([0.0]), np.array([lng]))
    assert int(ids[0]) == (0 << 61) | (d << 1) | 1
    # the same leaf on the v axis: lat = atan(v) at lng = 0 gives (i, j) =
    # (2^29, 3 * 2^28) on face 0
    face, _, _, s, t = C.project(np.array([np.degrees(np.arctan(u))]), np.array([0.0]))
    i, j = C.leaf_ij(s, t)
    assert face[0] == 0 and (int(i[0]), int(j[0])) == (1 << 29, 3 << 28)
