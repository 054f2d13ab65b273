"""CPU tests of the HIP library's host side (no GPU compute): symbol exports,
the index builder's structure and conservativeness, the lookup-table
encoding of Fig. 7b, the fp32 refinement tier's error bound, error paths."""
import os
import re
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import cellid as C

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def act():
    import paper_1802_09488_amd as act
    return act


def test_exports_every_declared_symbol(act):
    hdr = open(os.path.join(ROOT, "include", "act.h")).read()
    names = set(re.findall(r"\b(act_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 14
    for n in sorted(names):
        assert hasattr(act.lib, n), n
    assert act.version().startswith("act-mi355x")


def test_struct_layouts_match_the_header(act):
    import ctypes
    from paper_1802_09488_amd import _binding as B
    sz = (ctypes.c_int64 * 3)()
    assert B.lib.act_abi_sizes(sz) == 0
    assert list(sz) == [ctypes.sizeof(B.BuildOpts), ctypes.sizeof(B.JoinArgs),
                        ctypes.sizeof(B.Stats)]


def _decode(entry, lut):
    """(polygon id, interior) references of a tagged trie entry."""
    e = int(entry)
    tag = e & 3
    if e == 0:
        return []
    if tag == 1:
        v = [(e >> 2) & 0x7fffffff]
    elif tag == 2:
        v = [(e >> 2) & 0x7fffffff, (e >> 33) & 0x7fffffff]
    elif tag == 3:
        off = e >> 2
        nt = int(lut[off])
        v = [(int(x) << 1) | 1 for x in lut[off + 1:off + 1 + nt]]
        nc = int(lut[off + 1 + nt])
        v += [int(x) << 1 for x in lut[off + 2 + nt:off + 2 + nt + nc]]
    else:
        raise AssertionError("pointer entry returned by a lookup")
    return [(x >> 1, x & 1) for x in v]


def _truth(res):
    t = {}
    for i, o in enumerate(res.out):
        if o >= 0:
            t.setdefault(i, set()).add(int(o))
    for i, p in res.pairs:
        t.setdefault(int(i), set()).add(int(p))
    return t


def _structural_check(act, P, idx, pts, precision_m=None):
    face, _, _, s, tt = C.project(pts[:, 0], pts[:, 1])
    i, j = C.leaf_ij(s, tt)
    ent = idx.lookup_host(face, i, j)
    lut = idx.lut_host()
    res = oracle.join(P, pts)
    truth = _truth(res)
    extra = []
    for i in range(len(pts)):
        refs = _decode(ent[i], lut)
        ids_i = {p for p, _ in refs}
        T = truth.get(i, set())
        # conservative: every covering polygon is referenced by the point's cell
        assert T <= ids_i, (i, T, refs)
        # true hits are true
        for p, interior in refs:
            if interior:
                assert p in T, (i, p)
            elif p not in T:
                extra.append((i, p))
    if precision_m is not None and extra:
        e = np.asarray(extra, dtype=np.int64)
        d = oracle.boundary_dist_pairs(P, pts, e)
        assert d.max() <= precision_m + 1e-6, d.max()
    return ent


def test_builder_c1_exact_structure(act):
    P = synth.workload_polygons("c1")
    idx = act.build(P, "exact", device=-1)
    st = idx.stats()
    assert st["n_polys"] == 16 and st["max_cell_level"] == 20
    # depth bound: ceil((max level - prefix level) / 4) node levels (Section III-C)
    lp = st["face_prefix_level"][4]
    assert lp >= 0 and st["max_depth"] <= -(-(20 - lp) // 4) <= 8
    pts = np.concatenate([synth.workload_points("c1", 0, 30000), P.verts])
    _structural_check(act, P, idx, pts)


def test_builder_c2_approx_guarantee(act):
    P = synth.workload_polygons("c2")
    idx = act.build(P, "approx", 4.0, device=-1)
    st = idx.stats()
    assert st["mode"] == 1 and st["max_cell_level"] >= 21
    pts = synth.workload_points("c2", 0, 20000)
    _structural_check(act, P, idx, pts, precision_m=4.0)


def test_lut_matches_fig7b_golden(act):
    rows = [l.split() for l in open(os.path.join(ROOT, "tests", "golden", "lut_fig7b.txt"))
            if l.strip() and not l.startswith("#")]
    lut = np.zeros(0, np.uint32)
    for _, off, tru, cand, words in rows:
        refs = [(int(x) << 1) | 1 for x in tru.split(",")] + [int(x) << 1 for x in cand.split(",")]
        entry, lut = act.encode_refs_host(refs, lut)
        assert entry & 3 == 3 and entry >> 2 == int(off)
        w = [int(x) for x in words.split(",")]
        assert lut[int(off):int(off) + len(w)].tolist() == w
    # identical lists are stored once
    entry, lut2 = act.encode_refs_host([(5 << 1) | 1, 3 << 1, 1 << 1], lut)
    assert entry >> 2 == 0 and len(lut2) == len(lut)


def test_inline_payload_encoding(act):
    e, lut = act.encode_refs_host([(7 << 1) | 1])
    assert e & 3 == 1 and (e >> 2) == (7 << 1) | 1 and len(lut) == 0
    e, lut = act.encode_refs_host([(9 << 1), (3 << 1) | 1])
    assert e & 3 == 2 and ((e >> 2) & 0x7fffffff) == (3 << 1) | 1 and (e >> 33) == 9 << 1
    big = (1 << 30) - 1
    e, _ = act.encode_refs_host([(big << 1) | 1, (big - 1) << 1])
    assert (e >> 33) == (big << 1) | 1


@pytest.mark.parametrize("wl", ["c1", "c2"])
def test_cell_local_records_match_oracle(act, wl):
    """The cell-local refinement record of every candidate (cell, polygon)
    pair met by the points decides ST_Covers exactly as the oracle does
    (points from the workload, polygon vertices, edge midpoints and points
    nudged one ulp around them)."""
    P = synth.workload_polygons(wl)
    idx = act.build(P, "exact", device=-1)
    assert idx.stats()["local_words"] > 0
    rng = np.random.default_rng(23)
    v = P.verts[rng.choice(len(P.verts), min(len(P.verts), 3000), replace=False)]
    nudged = v + rng.integers(-1, 2, v.shape) * np.spacing(v)
    pts = np.concatenate([synth.workload_points(wl, 0, 3000), v, nudged])
    face, _, _, s, tt = C.project(pts[:, 0], pts[:, 1])
    i, j = C.leaf_ij(s, tt)
    ent = idx.lookup_host(face, i, j)
    lut = idx.lut_host()
    checked = 0
    for k in range(len(pts)):
        for p, interior in _decode(ent[k], lut):
            if interior:
                continue
            got = idx.refine_local_host(face[k], i[k], j[k], pts[k, 0], pts[k, 1], p)
            assert got == oracle.covers(P, p, pts[k, 0], pts[k, 1]), (k, p, pts[k])
            checked += 1
    assert checked > 1000


def _frac_sign(a, b, p):
    ax, ay, bx, by, px, py = (Fraction(float(v)) for v in (*a, *b, *p))
    d = (bx - ax) * (py - ay) - (by - ay) * (px - ax)
    return (d > 0) - (d < 0)


def _fp32_cases(rng, n):
    """(rows, origins, m_poly): near-degenerate lat/lng orientation tests of
    a polygon with origin o (points within 1e-16 .. 1e-6 degrees of an
    edge, edges from 1e-7 to 1e-3 degrees long)."""
    o = np.stack([rng.uniform(-74.2, -73.7, n), rng.uniform(40.5, 40.9, n)], 1)
    a = o + rng.uniform(-0.05, 0.05, (n, 2))
    b = a + rng.uniform(-1e-3, 1e-3, (n, 2)) * 10.0 ** rng.integers(-4, 1, (n, 1))
    t = rng.uniform(-0.2, 1.2, (n, 1))
    off = rng.uniform(-1, 1, (n, 2)) * 10.0 ** rng.integers(-16, -5, (n, 1))
    p = a + t * (b - a) + off
    m = np.max(np.abs(np.concatenate([(a - o), (b - o)], 1).astype(np.float32)), 1)
    return np.concatenate([a, b, p], 1), o, m


def test_fp32_tier_never_decides_wrong(act):
    """Invariant fuzz of the fp32 tier's error bound over 1e7 near-degenerate
    cases: whenever it decides, the sign equals the exact one (the oracle's
    exact sign, pinned against integer arithmetic in test_oracle.py; the
    first 20,000 decided cases also against fractions.Fraction)."""
    rng = np.random.default_rng(21)
    decided = fr = 0
    n = 10_000_000
    for c0 in range(0, n, 1_000_000):
        rows, o, m = _fp32_cases(rng, 1_000_000)
        # rows are (x, y) = (lng, lat) pairs; the tier sees them the same way
        got = act.orient_host_n(rows, 1, o, m)
        want = oracle.orient_signs(rows)
        dec = got != 0
        decided += int(dec.sum())
        bad = np.nonzero(dec & (got != want))[0]
        assert bad.size == 0, (rows[bad[:3]], o[bad[:3]], m[bad[:3]])
        if fr < 20000:
            for k in np.nonzero(dec)[0][:20000 - fr]:
                assert got[k] == _frac_sign(rows[k, 0:2], rows[k, 2:4], rows[k, 4:6])
                fr += 1
    assert decided > n // 10 and decided < n  # both outcomes occur
    # the single-call entry gives the same decisions
    rows, o, m = _fp32_cases(np.random.default_rng(5), 3000)
    got = act.orient_host_n(rows, 1, o, m)
    for k in range(3000):
        assert act.orient_fp32_host(rows[k, 0:2], rows[k, 2:4], rows[k, 4:6], o[k], m[k]) == got[k]


def test_exact_orient_matches_rationals(act):
    """The library's exact orientation (the builder's predicates and the last
    refinement tier) on 1e6 near-collinear cases and the oracle's adversarial
    set equals the oracle's pinned exact sign (and Fraction on 20,000)."""
    from test_oracle import adversarial_triples
    rng = np.random.default_rng(22)
    n = 500_000
    a = rng.uniform(-75, -73, (n, 2))
    b = rng.uniform(-75, -73, (n, 2))
    p = a + rng.uniform(-1, 2, (n, 1)) * (b - a) + rng.integers(-2, 3, (n, 2)) * np.spacing(a)
    rows = np.concatenate([np.concatenate([a, b, p], 1), adversarial_triples(rng, 500_000)])
    got = act.orient_host_n(rows, 0)
    want = oracle.orient_signs(rows)
    bad = np.nonzero(got != want)[0]
    assert bad.size == 0, rows[bad[:3]]
    assert (want == 0).sum() > 10000
    for k in range(0, 1_000_000, 50):
        assert got[k] == _frac_sign(rows[k, 0:2], rows[k, 2:4], rows[k, 4:6])
    for k in range(2000):
        assert act.orient_exact_host(rows[k, 0:2], rows[k, 2:4], rows[k, 4:6]) == got[k]


def _raw_build(act, verts, ring_off, poly_ring_off, mode=0, prec=0.0, device=-1):
    import ctypes
    from paper_1802_09488_amd import _binding as B
    v = np.ascontiguousarray(verts, dtype=np.float64)
    ro = np.ascontiguousarray(ring_off, dtype=np.int64)
    pro = np.ascontiguousarray(poly_ring_off, dtype=np.int32)
    opts = B.BuildOpts(max_level=0, device=device, threads=1, prefix_level=-1, margin_deg=0.0)
    h = ctypes.c_void_p()
    rc = B.lib.act_build(v.ctypes.data, ro.ctypes.data, pro.ctypes.data, len(pro) - 1, mode, prec,
                         ctypes.byref(opts), ctypes.byref(h))
    if rc == 0:
        B.lib.act_free(h)
    return rc


def test_build_is_deterministic(act):
    """The index image does not depend on the build's thread count."""
    P = synth.workload_polygons("c1")
    for mode, prec in (("exact", 0.0), ("approx", 4.0)):
        d1 = act.build(P, mode, prec, device=-1, threads=1).digest()
        d8 = act.build(P, mode, prec, device=-1, threads=8).digest()
        d8b = act.build(P, mode, prec, device=-1, threads=8).digest()
        assert d1 == d8 == d8b


def test_error_paths(act):
    from paper_1802_09488_amd import _binding as B
    sq = np.array([[0, 0], [0, 1], [1, 1], [1, 0]], float)
    assert _raw_build(act, sq, [0, 4], [0, 1]) == 0
    assert _raw_build(act, sq[:2], [0, 2], [0, 1]) == B.ACT_E_POLY          # < 3 vertices
    assert _raw_build(act, np.array([[0, 0], [0, 0], [0, 0], [1, 1]], float),
                      [0, 4], [0, 1]) == B.ACT_E_POLY                        # duplicates only
    bad = sq.copy()
    bad[1, 0] = np.nan
    assert _raw_build(act, bad, [0, 4], [0, 1]) == B.ACT_E_POLY            # NaN vertex
    bad = sq.copy()
    bad[1, 1] = 200.0
    assert _raw_build(act, bad, [0, 4], [0, 1]) == B.ACT_E_POLY            # lng out of range
    assert _raw_build(act, sq, [0, 4], [0, 1], mode=7) == B.ACT_E_ARG
    assert _raw_build(act, sq, [0, 4], [0, 1], mode=1, prec=0.001) == B.ACT_E_ARG
    assert _raw_build(act, sq, [0, 4], [0, 0]) == B.ACT_E_POLY             # polygon w/o ring
    # joins on a host-only index are refused before anything is launched
    P = synth.Polygons.from_rings([[sq]])
    idx = act.build(P, "exact", device=-1)
    rc = B.lib.act_join(idx.handle, None, 10, None, None)
    assert rc == B.ACT_E_DEVICE
    assert b"without a device" in B.lib.act_last_error()
    assert B.lib.act_join(None, None, 0, None, None) == B.ACT_E_ARG


def test_empty_polygon_set(act):
    P = synth.Polygons(np.zeros((0, 2)), np.zeros(1, np.int64), np.zeros(1, np.int32))
    idx = act.build(P, "exact", device=-1)
    st = idx.stats()
    assert st["n_cells"] == 0 and st["n_faces"] == 0
    assert idx.lookup_host([4], [5], [7]).tolist() == [0]


def _cand_fraction(idx, pts):
    """Share of points whose cell has a candidate reference (host lookups)."""
    face, _, _, s, tt = C.project(pts[:, 0], pts[:, 1])
    i, j = C.leaf_ij(s, tt)
    ent = idx.lookup_host(face, i, j)
    lut = idx.lut_host()
    return np.mean([any(not inter for _, inter in _decode(e, lut)) for e in ent])


def test_training_refines_expensive_cells(act):
    """Training (Section III-D) with points of the workload's distribution:
    cells are split, the index stays conservative (every covering polygon
    referenced, interior references true, checked against the oracle on
    fresh points and on the training points), fewer fresh points land in
    expensive cells, and the build is deterministic."""
    P = synth.workload_polygons("c2")
    tp = synth.training_points("c2", 300_000)
    base = act.build(P, "exact", device=-1, max_level=16)
    idx = act.build(P, "exact", device=-1, max_level=16, train_points=tp)
    st = idx.stats()
    assert st["train_splits"] > 1000 and st["train_points_used"] == len(tp)
    assert st["max_cell_level"] > 16 and st["n_cells"] > base.stats()["n_cells"]
    pts = np.concatenate([synth.workload_points("c2", 0, 20000), tp[:5000], P.verts[::7]])
    _structural_check(act, P, idx, pts)
    fresh = synth.workload_points("c2", 50_000, 70_000)
    assert _cand_fraction(idx, fresh) < 0.8 * _cand_fraction(base, fresh)
    again = act.build(P, "exact", device=-1, max_level=16, train_points=tp, threads=3)
    assert again.digest() == idx.digest()
    # the local records of split cells decide like the oracle
    face, _, _, s, tt = C.project(pts[:, 0], pts[:, 1])
    i, j = C.leaf_ij(s, tt)
    ent = idx.lookup_host(face, i, j)
    lut = idx.lut_host()
    checked = 0
    for k in range(0, len(pts), 3):
        for p, interior in _decode(ent[k], lut):
            if not interior:
                got = idx.refine_local_host(face[k], i[k], j[k], pts[k, 0], pts[k, 1], p)
                assert got == oracle.covers(P, p, pts[k, 0], pts[k, 1])
                checked += 1
    assert checked > 100


def test_training_respects_memory_budget(act):
    """Training stops when the next split would take the device image past
    the budget: the image stays within it and not every training point was
    used; a budget below the untrained image trains nothing; approximate
    indexes ignore training."""
    P = synth.workload_polygons("c2")
    tp = synth.training_points("c2", 300_000)
    base = act.build(P, "exact", device=-1, max_level=16).stats()
    budget = base["image_bytes"] + 200_000
    st = act.build(P, "exact", device=-1, max_level=16, train_points=tp,
                   memory_budget=budget).stats()
    assert 0 < st["train_splits"] and st["train_points_used"] < len(tp)
    assert base["image_bytes"] < st["image_bytes"] <= budget
    st0 = act.build(P, "exact", device=-1, max_level=16, train_points=tp,
                    memory_budget=base["image_bytes"] - 1).stats()
    assert st0["train_splits"] == 0 and st0["image_bytes"] == base["image_bytes"]
    sa = act.build(P, "approx", 8.0, device=-1, train_points=tp).stats()
    assert sa["train_splits"] == 0
    cap = act.build(P, "exact", device=-1, max_level=16, train_points=tp,
                    train_max_level=17).stats()
    assert cap["max_cell_level"] == 17


def test_auto_policy_follows_the_budget(act):
    """ACT_AUTO (Section III-A): the approximate index when it fits the
    budget; else the exact index, its covering level lowered until the
    untrained image fits, then trained within the budget; an error when
    nothing fits."""
    P = synth.workload_polygons("c2")
    tp = synth.training_points("c2", 200_000)
    approx = act.build(P, "approx", 4.0, device=-1).stats()
    big = act.build(P, "auto", 4.0, device=-1, memory_budget=approx["image_bytes"],
                    train_points=tp)
    assert big.mode == act.ACT_APPROX and big.stats()["image_bytes"] == \
        approx["image_bytes"]
    budget = approx["image_bytes"] - 1
    small = act.build(P, "auto", 4.0, device=-1, memory_budget=budget, train_points=tp)
    st = small.stats()
    assert small.mode == act.ACT_EXACT and st["image_bytes"] <= budget
    assert st["train_splits"] > 0
    pts = synth.workload_points("c2", 0, 5000)
    _structural_check(act, P, small, pts)
    with pytest.raises(act.ActError) as e:
        act.build(P, "auto", 4.0, device=-1, memory_budget=100_000)
    assert e.value.code == -7
    with pytest.raises(act.ActError):
        act.build(P, "auto", 4.0, device=-1)  # no budget


def test_save_load_roundtrip(act, tmp_path):
    """An index file reproduces the index (digest, statistics, lookups); a
    corrupt, truncated or foreign file is refused."""
    P = synth.workload_polygons("c2")
    for mode, prec, kw in (("exact", 0.0, {"train_points": synth.training_points("c2", 50_000)}),
                           ("approx", 4.0, {})):
        idx = act.build(P, mode, prec, device=-1, **kw)
        path = tmp_path / ("%s.act" % mode)
        idx.save(path)
        got = act.load(path, device=-1)
        assert got.digest() == idx.digest()
        a, b = idx.stats(), got.stats()
        for k in ("n_cells", "n_nodes", "lut_words", "local_words", "max_depth", "mode",
                  "precision_m", "train_splits", "image_bytes", "face_prefix_level"):
            assert a[k] == b[k], k
        pts = synth.workload_points("c2", 0, 20000)
        face, _, _, s, tt = C.project(pts[:, 0], pts[:, 1])
        i, j = C.leaf_ij(s, tt)
        assert np.array_equal(idx.lookup_host(face, i, j), got.lookup_host(face, i, j))
    raw = bytearray(path.read_bytes())
    for label, data in (("flip", raw[:1000] + bytes([raw[1000] ^ 1]) + raw[1001:]),
                        ("truncated", raw[:-9]), ("foreign", b"not an index" + raw[12:])):
        bad = tmp_path / ("bad_%s.act" % label)
        bad.write_bytes(bytes(data))
        with pytest.raises(act.ActError) as e:
            act.load(bad, device=-1)
        assert e.value.code == -1, label
    with pytest.raises(act.ActError):
        act.load(tmp_path / "missing.act", device=-1)


def _fnv(data: bytes) -> int:
    d = 0xcbf29ce484222325
    for b in data:
        d = ((d ^ b) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    return d


def test_load_refuses_out_of_range_references(act, tmp_path):
    """A file whose digest is right but whose trie points outside the image
    (a child pointer past the last node, a list offset past the table) is
    refused: the loader checks every reference the probe would follow."""
    import struct
    sq = [np.array([[40.70, -74.00], [40.70, -73.99], [40.71, -73.99], [40.71, -74.00]])]
    P = synth.Polygons.from_rings([sq])
    idx = act.build(P, "exact", device=-1)
    path = tmp_path / "sq.act"
    idx.save(path)
    raw = bytearray(path.read_bytes())
    assert _fnv(bytes(raw[:-8])) == struct.unpack("<Q", raw[-8:])[0]  # the documented digest
    assert act.load(path, device=-1).digest() == idx.digest()
    # magic, version, extra bytes (16), the scalars (220), then the node
    # array's length and entries
    at = 16 + 220
    n_nodes = struct.unpack("<Q", raw[at:at + 8])[0] // 256
    ent = np.frombuffer(bytes(raw[at + 8:at + 8 + 8 * 256 * n_nodes]), dtype=np.uint64)
    for label, want_tag, value in (("pointer", 0, (n_nodes + 5) << 2),
                                   ("list", 3, ((1 << 29) << 2) | 3)):
        k = int(np.nonzero((ent != 0) & ((ent & np.uint64(3)) == np.uint64(want_tag)))[0][0])
        bad = bytearray(raw)
        bad[at + 8 + 8 * k:at + 16 + 8 * k] = struct.pack("<Q", value)
        bad[-8:] = struct.pack("<Q", _fnv(bytes(bad[:-8])))
        p = tmp_path / ("bad_%s.act" % label)
        p.write_bytes(bytes(bad))
        with pytest.raises(act.ActError) as e:
            act.load(p, device=-1)
        assert "corrupt" in str(e.value), label


def test_sphere_index_structure(act, tmp_path):
    """Spherical geometry (great-circle edges): the cell margin grows by the
    largest arc-to-chord distance, and the index stays conservative for the
    arcs: every polygon that covers a point in the spherical model (oracle)
    is referenced by the point's cell and every true hit is a spherical
    containment; approximate mode refuses it; index files keep it."""
    P = synth.workload_polygons("c2")
    idx = act.build(P, "exact", device=-1, geometry="sphere")
    st = idx.stats()
    assert st["geometry"] == 1 and st["margin_deg"] > 1e-9
    assert act.build(P, "exact", device=-1).stats()["margin_deg"] == 1e-9
    rng = np.random.default_rng(29)
    v = P.verts[rng.choice(len(P.verts), 3000, replace=False)]
    pts = np.concatenate([synth.workload_points("c2", 0, 20000), v,
                          v + rng.integers(-2, 3, v.shape) * np.spacing(v)])
    face, _, _, s, tt = C.project(pts[:, 0], pts[:, 1])
    i, j = C.leaf_ij(s, tt)
    ent = idx.lookup_host(face, i, j)
    lut = idx.lut_host()
    truth = _truth(oracle.join_sphere(P, pts))
    for k in range(len(pts)):
        refs = _decode(ent[k], lut)
        ids_k = {p for p, _ in refs}
        assert truth.get(k, set()) <= ids_k, (k, truth.get(k), refs)
        for p, interior in refs:
            if interior:
                assert p in truth.get(k, set()), (k, p)
    with pytest.raises(act.ActError):
        act.build(P, "approx", 4.0, device=-1, geometry="sphere")
    path = tmp_path / "sphere.act"
    idx.save(path)
    got = act.load(path, device=-1)
    assert got.digest() == idx.digest() and got.stats()["geometry"] == 1


def test_budgeted_coverings(act):
    """Per-polygon coverings with the paper's cell budgets (128 covering
    cells up to level 30, 256 interior cells up to level 20), merged without
    overlap: the index is conservative against the oracle (every covering
    polygon referenced, every true hit true), far smaller than the joint
    subdivision, and training with points of the workload's distribution
    makes more points solely true hits (the Table IV effect)."""
    P = synth.workload_polygons("c2")
    idx = act.build(P, "exact", device=-1, max_level=30, max_covering_cells=128)
    st = idx.stats()
    joint = act.build(P, "exact", device=-1).stats()
    assert st["n_cells"] < joint["n_cells"] / 4 and st["n_nodes"] < joint["n_nodes"] / 4
    rng = np.random.default_rng(31)
    v = P.verts[rng.choice(len(P.verts), 2000, replace=False)]
    pts = np.concatenate([synth.workload_points("c2", 0, 20000), v,
                          v + rng.integers(-1, 2, v.shape) * np.spacing(v)])
    _structural_check(act, P, idx, pts)
    trained = act.build(P, "exact", device=-1, max_level=30, max_covering_cells=128,
                        train_points=synth.training_points("c2", 300_000))
    assert trained.stats()["train_splits"] > 1000
    _structural_check(act, P, trained, pts[:5000])
    fresh = synth.workload_points("c2", 50_000, 70_000)
    assert _cand_fraction(trained, fresh) < 0.7 * _cand_fraction(idx, fresh)
    with pytest.raises(act.ActError):
        act.build(P, "approx", 4.0, device=-1, max_covering_cells=128)
