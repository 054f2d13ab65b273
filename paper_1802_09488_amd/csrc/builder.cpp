// builder.cpp -- host construction of the logical and physical index.
//
// Logical index (Section III-B): the paper computes per-polygon coverings
// and interior coverings and merges them into a super covering whose cells
// never overlap, keeping each cell's (polygon id, interior flag) references
// (flavour (iii), Listing 1, Fig. 5). Here the coverings of all polygons are
// computed jointly by one recursive subdivision of the six cube faces: a
// cell is classified against every polygon that can reach it as INTERIOR
// (cell inside the polygon), EXTERIOR (disjoint) or BOUNDARY (an edge meets
// the cell). Recursion stops when no polygon is BOUNDARY, at the maximum
// covering level (exact mode), or once the cell's diagonal is below the
// requested precision (approximate mode, Section III-A). The emitted cells
// are disjoint by construction and carry exactly the references a merge of
// the individual coverings with precision-preserving conflict resolution
// would give them.
//
// Classification is conservative so that exact-mode output is bit-exact:
// every cell is represented by a lat/lng box that contains the cell's
// region on the sphere (corner points plus the latitude extremes of its
// great-circle edges), inflated by a margin that dominates the GPU's fp64
// projection rounding. All predicates on that box are exact (geom.hpp).
//
// Exact mode adds, per candidate (cell, polygon), a cell-local refinement
// record (see local_record) so that a candidate point need not be tested
// against all of the polygon's edges.
//
// Physical index (Section III-C): cells are denormalised to the node levels
// of their face (g = 4 levels per node, Fig. 7a), references of fewer than
// three polygons are inlined into the tagged entry, longer lists are
// deduplicated into the lookup table (Fig. 7b). The trie is keyed by each
// cell's quadtree path (see index.hpp).
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <string>
#include <thread>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "cellid.hpp"
#include "geom.hpp"
#include "index.hpp"

namespace act {

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kDeg = 180.0 / kPi;
constexpr double kEarthR = 6371008.8;

// Lat/lng box. When `wrap` is set the longitude range crosses the
// antimeridian and consists of the two pieces [lng0, 180] and [-180, lng1].
struct Box {
  double lat0, lat1, lng0, lng1;
  bool wrap = false;
  int pieces() const { return wrap ? 2 : 1; }
  double plo(int k) const { return wrap ? (k == 0 ? lng0 : -180.0) : lng0; }
  double phi(int k) const { return wrap ? (k == 0 ? 180.0 : lng1) : lng1; }
};

struct Prep {
  int n_polys = 0;
  std::vector<int32_t> e_off;    // per polygon edge range
  std::vector<double> ex;        // edges: ax ay bx by (x = lng, y = lat)
  std::vector<Box> bbox;         // per polygon
};

// ---------------------------------------------------------------- geometry

void face_uv_xyz(int face, double u, double v, double c[3]) {
  int a = face % 3;
  c[a] = face >= 3 ? -1.0 : 1.0;
  c[(a + 1) % 3] = u;
  c[(a + 2) % 3] = v;
}

double lat_of(const double c[3]) { return std::atan2(c[2], std::hypot(c[0], c[1])) * kDeg; }
double lng_of(const double c[3]) { return std::atan2(c[1], c[0]) * kDeg; }

void cross3(const double a[3], const double b[3], double o[3]) {
  o[0] = a[1] * b[2] - a[2] * b[1];
  o[1] = a[2] * b[0] - a[0] * b[2];
  o[2] = a[0] * b[1] - a[1] * b[0];
}
double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// Lat/lng bounds of the cell's region (no margin). The region is bounded by
// four great-circle arcs: latitude can peak inside an arc (the point of the
// arc's circle closest to a pole), longitude is monotone along each arc and
// sweeps less than 180 degrees, so unless the cell holds a pole its longitude
// range is the smallest circular interval containing the corners (which may
// cross the antimeridian). Cells spanning more than 90 degrees of longitude
// get the full range.
Box cell_bounds(int face, int level, uint32_t i, uint32_t j) {
  double inv = std::ldexp(1.0, -level);
  double u0 = uv_from_st(i * inv), u1 = uv_from_st((i + 1) * inv);
  double v0 = uv_from_st(j * inv), v1 = uv_from_st((j + 1) * inv);
  double P[4][3];
  face_uv_xyz(face, u0, v0, P[0]);
  face_uv_xyz(face, u1, v0, P[1]);
  face_uv_xyz(face, u1, v1, P[2]);
  face_uv_xyz(face, u0, v1, P[3]);
  Box b{90, -90, 180, -180};
  double lng[4];
  for (int k = 0; k < 4; k++) {
    double la = lat_of(P[k]);
    lng[k] = lng_of(P[k]);
    b.lat0 = std::min(b.lat0, la);
    b.lat1 = std::max(b.lat1, la);
  }
  for (int k = 0; k < 4; k++) {
    const double *A = P[k], *B = P[(k + 1) & 3];
    double n[3];
    cross3(A, B, n);
    double nxy2 = n[0] * n[0] + n[1] * n[1];
    if (nxy2 <= 0) continue;
    double m[3] = {-n[0] * n[2], -n[1] * n[2], nxy2};
    for (int sgn = -1; sgn <= 1; sgn += 2) {
      double q[3] = {sgn * m[0], sgn * m[1], sgn * m[2]};
      double t1[3], t2[3];
      cross3(A, q, t1);
      cross3(q, B, t2);
      if (dot3(t1, n) >= 0 && dot3(t2, n) >= 0) {
        double la = lat_of(q);
        b.lat0 = std::min(b.lat0, la);
        b.lat1 = std::max(b.lat1, la);
      }
    }
  }
  bool pole = (face % 3 == 2) && u0 <= 0 && u1 >= 0 && v0 <= 0 && v1 >= 0;
  if (pole) {
    if (face == 2) b.lat1 = 90;
    else b.lat0 = -90;
    b.lng0 = -180;
    b.lng1 = 180;
    return b;
  }
  // smallest circular interval holding the four corner longitudes
  std::sort(lng, lng + 4);
  double gap = lng[0] + 360.0 - lng[3];
  int after = 0;  // index of the value right after the largest gap
  for (int k = 1; k < 4; k++)
    if (lng[k] - lng[k - 1] > gap) {
      gap = lng[k] - lng[k - 1];
      after = k;
    }
  if (360.0 - gap > 90.0) {
    b.lng0 = -180;
    b.lng1 = 180;
  } else if (after == 0) {
    b.lng0 = lng[0];
    b.lng1 = lng[3];
  } else {
    b.lng0 = lng[after];
    b.lng1 = lng[after - 1];
    b.wrap = true;
  }
  return b;
}

// Inflate by the margin. A child's box is not clipped to its parent's: the
// child's region lies inside the parent's, so classifying the child only
// against the edges that meet the parent box decides the child box's part
// inside the parent box, which still holds the child region plus nearly the
// whole margin.
Box inflate(Box b, double margin) {
  b.lat0 -= margin;
  b.lat1 += margin;
  b.lng0 -= margin;
  b.lng1 += margin;
  if (!b.wrap && b.lng1 - b.lng0 >= 360.0) {
    b.lng0 = -180 - margin;
    b.lng1 = 180 + margin;
  }
  return b;
}

// Upper bound of the planar distance (local equirectangular frame at any
// latitude of the box) between two points of the box, in metres.
double box_diag_m(const Box &b) {
  double k = kEarthR * kPi / 180.0;
  double maxcos = (b.lat0 <= 0 && b.lat1 >= 0)
                      ? 1.0
                      : std::cos(std::min(std::fabs(b.lat0), std::fabs(b.lat1)) / kDeg);
  // the planar model does not wrap: a box across the antimeridian is as wide
  // as the plane
  double w = b.wrap ? 360.0 : b.lng1 - b.lng0;
  double dx = w * maxcos, dy = b.lat1 - b.lat0;
  // small relative slack for rounding in this evaluation
  return k * std::sqrt(dx * dx + dy * dy) * (1.0 + 1e-12);
}

// Cell box (possibly wrapped) vs a polygon's bounding box (never wrapped).
bool boxes_meet(const Box &a, const Box &pb) {
  if (a.lat1 < pb.lat0 || pb.lat1 < a.lat0) return false;
  for (int k = 0; k < a.pieces(); k++)
    if (!(a.phi(k) < pb.lng0 || pb.lng1 < a.plo(k))) return true;
  return false;
}

bool segment_meets(const double *q, const Box &b) {
  for (int k = 0; k < b.pieces(); k++)
    if (segment_meets_box(q[0], q[1], q[2], q[3], b.plo(k), b.phi(k), b.lat0, b.lat1)) return true;
  return false;
}

bool poly_covers(const Prep &P, int p, double x, double y) {
  int inside = 0;
  for (int e = P.e_off[p]; e < P.e_off[p + 1]; e++) {
    const double *q = &P.ex[4 * (size_t)e];
    int r = edge_test_exact(q[0], q[1], q[2], q[3], x, y);
    if (r == 2) return true;
    inside ^= r;
  }
  return inside != 0;
}

// ------------------------------------------------------------ subdivision

struct Bref {
  int32_t poly, off, cnt;  // edges[off .. off+cnt) meet the cell's box
};

struct Work {
  int face, level;
  uint32_t i, j;
  Box box;
  std::vector<int32_t> interior;  // polygons containing the cell
  std::vector<Bref> bnd;
  std::vector<int32_t> edges;
};

struct CellOut {
  int32_t face, level;
  uint32_t i, j;  // coordinates at the cell's level
  int32_t ref_off, ref_cnt;
};

struct Sink {
  std::vector<CellOut> cells;
  std::vector<uint32_t> refs;  // id << 1 | interior
  std::vector<uint32_t> locs;  // per ref: local record offset in `local` (candidates)
  std::vector<uint32_t> local; // cell-local refinement records (exact mode)
};

struct Ctx {
  const Prep *P;
  BuildParams bp;
  std::atomic<bool> failed{false};
  std::string err;
  int err_code = ACT_E_ARG;
  std::atomic<int64_t> cells_out{0};  // cells emitted so far (for bp.cell_limit)
};

// Classify a child box given the parent's candidates.
void classify(const Ctx &C, const Box &box, const std::vector<int32_t> &pint,
              const std::vector<Bref> &pbnd, const std::vector<int32_t> &pedges, Work &w) {
  const Prep &P = *C.P;
  w.interior = pint;
  w.bnd.clear();
  w.edges.clear();
  for (const Bref &br : pbnd) {
    if (!boxes_meet(box, P.bbox[br.poly])) continue;
    int32_t off = (int32_t)w.edges.size();
    for (int k = 0; k < br.cnt; k++) {
      int e = pedges[br.off + k];
      const double *q = &P.ex[4 * (size_t)e];
      if (segment_meets(q, box)) w.edges.push_back(e);
    }
    int32_t cnt = (int32_t)w.edges.size() - off;
    if (cnt > 0) {
      w.bnd.push_back({br.poly, off, cnt});
    } else {
      // no edge meets the box: each (convex) piece is inside or outside
      double cy = 0.5 * (box.lat0 + box.lat1);
      int in = 0;
      for (int k = 0; k < box.pieces(); k++)
        in += poly_covers(P, br.poly, 0.5 * (box.plo(k) + box.phi(k)), cy);
      if (in == box.pieces()) w.interior.push_back(br.poly);
      else if (in > 0) w.bnd.push_back({br.poly, off, 0});  // undecided: keep as candidate
    }
  }
  std::sort(w.interior.begin(), w.interior.end());
}

// Cell-local refinement record of polygon p for a cell with box b (exact
// mode). For a point q inside b, the ray from q towards +x crosses
//   * edges that meet b: tested exactly at probe time (stored);
//   * edges that do not meet b: within b's latitude band such an edge lies
//     wholly left or wholly right of b; a right one is crossed exactly when
//     it straddles q's latitude, [ylo <= q.y] xor [yhi <= q.y] with the
//     half-open rule. Their parity is stored as a base bit (breakpoints at
//     or below the band's bottom) plus the sorted breakpoints inside the
//     band. Edges outside the band and horizontal edges never contribute.
// Layout (32-bit words, doubles 8-byte aligned): n_local, n_break | base << 31,
// n_local x (ax, ay, bx, by), n_break breakpoints ascending.
static uint32_t local_record(const Prep &P, int p, const Box &b, std::vector<uint32_t> &out) {
  std::vector<double> loc, brk;
  int base = 0;
  for (int e = P.e_off[p]; e < P.e_off[p + 1]; e++) {
    const double *q = &P.ex[4 * (size_t)e];
    if (b.wrap || segment_meets(q, b)) {  // boxes across the antimeridian keep every edge
      loc.insert(loc.end(), q, q + 4);
      continue;
    }
    const bool up = q[1] <= q[3];
    const double lx = up ? q[0] : q[2], ly = up ? q[1] : q[3];
    const double ux = up ? q[2] : q[0], uy = up ? q[3] : q[1];
    if (ly == uy || uy < b.lat0 || ly > b.lat1) continue;
    const double ys = std::max(ly, b.lat0);
    if (orient_sign_exact(lx, ly, ux, uy, b.lng1, ys) <= 0) continue;  // left of the box
    for (double y : {ly, uy}) {
      if (y <= b.lat0) base ^= 1;
      else if (y <= b.lat1) brk.push_back(y);
    }
  }
  std::sort(brk.begin(), brk.end());
  const uint32_t off = (uint32_t)out.size();
  out.push_back((uint32_t)(loc.size() / 4));
  out.push_back((uint32_t)brk.size() | ((uint32_t)base << 31));
  auto put = [&](double v) {
    uint32_t w[2];
    std::memcpy(w, &v, 8);
    out.push_back(w[0]);
    out.push_back(w[1]);
  };
  for (double v : loc) put(v);
  for (double v : brk) put(v);
  return off;
}

void emit(Ctx &C, const Work &w, Sink &s) {
  if (C.bp.cell_limit > 0 && C.cells_out.fetch_add(1, std::memory_order_relaxed) >= C.bp.cell_limit &&
      !C.failed.exchange(true)) {
    C.err = "the covering exceeds the memory budget";
    C.err_code = ACT_E_RANGE;
  }
  CellOut c;
  c.face = w.face;
  c.level = w.level;
  c.i = w.i;
  c.j = w.j;
  c.ref_off = (int32_t)s.refs.size();
  size_t a = 0, b = 0;
  // merge interior (flag 1) and boundary (flag 0) ids in ascending order
  std::vector<int32_t> bids;
  bids.reserve(w.bnd.size());
  for (const Bref &br : w.bnd) bids.push_back(br.poly);
  std::sort(bids.begin(), bids.end());
  const bool local = C.bp.mode == ACT_EXACT && C.bp.geometry == ACT_GEOM_PLANE;
  while (a < w.interior.size() || b < bids.size()) {
    if (b >= bids.size() || (a < w.interior.size() && w.interior[a] < bids[b])) {
      s.refs.push_back(((uint32_t)w.interior[a++] << 1) | 1u);
      s.locs.push_back(UINT32_MAX);
    } else {
      s.refs.push_back((uint32_t)bids[b] << 1);
      s.locs.push_back(local ? local_record(*C.P, bids[b], w.box, s.local) : UINT32_MAX);
      b++;
    }
  }
  c.ref_cnt = (int32_t)s.refs.size() - c.ref_off;
  s.cells.push_back(c);
}

// Decide a cell: returns true if it must be split further.
bool settle(Ctx &C, const Work &w, Sink &s) {
  if (w.bnd.empty()) {
    if (!w.interior.empty()) emit(C, w, s);
    return false;
  }
  if (C.bp.mode == ACT_EXACT) {
    if (w.level >= C.bp.max_level) {
      emit(C, w, s);
      return false;
    }
    return true;
  }
  if (box_diag_m(w.box) < C.bp.precision_m) {
    emit(C, w, s);
    return false;
  }
  if (w.level >= kMaxLevel) {
    if (w.box.wrap) {  // level-30 cell on the antimeridian: emitted as is
      emit(C, w, s);
      return false;
    }
    if (!C.failed.exchange(true))
      C.err = "precision_m is below the diagonal of the finest (level-30) cell";
    return false;
  }
  return true;
}

void make_child(Ctx &C, const Work &w, int q, Work &c) {
  c.face = w.face;
  c.level = w.level + 1;
  c.i = (w.i << 1) | (uint32_t)(q >> 1);
  c.j = (w.j << 1) | (uint32_t)(q & 1);
  c.box = inflate(cell_bounds(c.face, c.level, c.i, c.j), C.bp.margin_deg);
  classify(C, c.box, w.interior, w.bnd, w.edges, c);
}

void dfs(Ctx &C, const Work &w, Sink &s) {
  if (C.failed.load(std::memory_order_relaxed)) return;
  if (!settle(C, w, s)) return;
  Work c;
  for (int q = 0; q < 4; q++) {
    make_child(C, w, q, c);
    dfs(C, c, s);
  }
}

// ------------------------------------- coverings with per-polygon cell budgets
//
// The paper computes a covering and an interior covering of each polygon
// with S2's region coverer under cell-count budgets (Section V: at most 128
// covering cells up to level 30, at most 256 interior cells up to level 20)
// and merges them into a super covering (Section III-B, flavour iii). Here
// each polygon's coverings are computed greedily, coarsest cells first:
//   covering: a cell inside the polygon is final; a boundary cell is
//   replaced by its children that meet the polygon while the cells kept,
//   queued and the new children stay within the budget (and the level cap),
//   else it is final. Every cell that meets the polygon stays covered.
//   interior covering: cells inside the polygon are kept; boundary cells
//   are expanded while the budget and the level cap allow, else dropped.
// Cell status is the conservative classification of the joint subdivision
// (exact tests on the cell's inflated box), for the one polygon.

struct CoverCell {
  int face, level;
  uint32_t i, j;
  bool interior;  // the cell lies inside the polygon
};

// Key of a cell (coordinates at its level): face, quadtree path (i above j
// at each level) and a marker bit, laid out like a cell id.
static uint64_t code_of(int face, int level, uint32_t i, uint32_t j) {
  uint64_t key = 0;
  for (int b = level - 1; b >= 0; b--) key = (key << 2) | (((i >> b) & 1u) << 1) | ((j >> b) & 1u);
  const int sh = 2 * (kMaxLevel - level);
  return ((uint64_t)face << 61) | (key << (sh + 1)) | (1ull << sh);
}

// One polygon's covering (interior = false) or interior covering.
static void cover_polygon(Ctx &C, int p, bool interior_only, int max_cells, int max_level,
                          std::vector<CoverCell> &out) {
  const Prep &P = *C.P;
  std::vector<Bref> bnd{{p, 0, P.e_off[p + 1] - P.e_off[p]}};
  std::vector<int32_t> edges;
  for (int e = P.e_off[p]; e < P.e_off[p + 1]; e++) edges.push_back(e);
  std::vector<int32_t> none;
  // the queue, coarsest first (ties: face, i, j), as a binary heap
  std::vector<Work> pool;
  auto worse = [&pool](size_t a, size_t b) {
    const Work &x = pool[a], &y = pool[b];
    if (x.level != y.level) return x.level > y.level;
    if (x.face != y.face) return x.face > y.face;
    return x.i != y.i ? x.i > y.i : x.j > y.j;
  };
  std::vector<size_t> heap;
  auto push = [&](Work &&w) {
    pool.push_back(std::move(w));
    heap.push_back(pool.size() - 1);
    std::push_heap(heap.begin(), heap.end(), worse);
  };
  auto met = [&](const Work &w) { return !w.interior.empty() || !w.bnd.empty(); };
  for (int face = 0; face < 6; face++) {
    Work w;
    w.face = face;
    w.level = 0;
    w.i = w.j = 0;
    w.box = inflate(cell_bounds(face, 0, 0, 0), C.bp.margin_deg);
    classify(C, w.box, none, bnd, edges, w);
    if (met(w)) push(std::move(w));
  }
  int kept = 0;
  while (!heap.empty()) {
    std::pop_heap(heap.begin(), heap.end(), worse);
    const size_t k = heap.back();
    heap.pop_back();
    const Work w = std::move(pool[k]);
    if (w.bnd.empty()) {  // inside the polygon
      out.push_back({w.face, w.level, w.i, w.j, true});
      kept++;
      continue;
    }
    Work ch[4];
    int n_ch = 0;
    if (w.level < max_level)
      for (int q = 0; q < 4; q++) {
        make_child(C, w, q, ch[n_ch]);
        if (met(ch[n_ch])) n_ch++;
      }
    const bool expand = w.level < max_level && kept + (int)heap.size() + n_ch <= max_cells;
    if (expand) {
      for (int q = 0; q < n_ch; q++) push(std::move(ch[q]));
    } else if (!interior_only) {
      out.push_back({w.face, w.level, w.i, w.j, false});
      kept++;
    }
  }
}

// The super covering of the polygons' budgeted coverings (flavour iii:
// no overlap, each cell keeps the references of every covering cell it
// lies in; a polygon is a true hit where one of its interior cells lies).
// Overlaps are resolved top-down: a cell with indexed descendants hands its
// references to its four children. Emits the cells into `sink`.
static void budget_super_covering(Ctx &C, int nthreads, Sink &sink) {
  const BuildParams &bp = C.bp;
  const int np = C.P->n_polys;
  std::vector<std::vector<CoverCell>> cov(np), inn(np);
  std::atomic<int> next{0};
  auto work = [&]() {
    for (int p; (p = next.fetch_add(1)) < np;) {
      cover_polygon(C, p, false, bp.max_covering_cells, bp.max_level, cov[p]);
      cover_polygon(C, p, true, bp.max_interior_cells, bp.max_interior_level, inn[p]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; t++) pool.emplace_back(work);
  work();
  for (auto &th : pool) th.join();
  // references of every indexed cell, and the set of proper ancestors
  std::unordered_map<uint64_t, std::vector<uint32_t>> own;
  std::unordered_set<uint64_t> above;
  for (int p = 0; p < np; p++)
    for (const auto *list : {&cov[p], &inn[p]})
      for (const CoverCell &c : *list) {
        own[code_of(c.face, c.level, c.i, c.j)].push_back(((uint32_t)p << 1) | (c.interior ? 1u : 0u));
        for (int l = c.level - 1; l >= 0; l--)
          if (!above.insert(code_of(c.face, l, c.i >> (c.level - l), c.j >> (c.level - l))).second)
            break;  // its ancestors are in already
      }
  cov.clear();
  inn.clear();
  // top-down: references inherited from covering ancestors
  struct Frame {
    int face, level;
    uint32_t i, j;
    std::vector<uint32_t> refs;
  };
  std::vector<Frame> stack;
  for (int face = 5; face >= 0; face--) stack.push_back({face, 0, 0, 0, {}});
  while (!stack.empty()) {
    Frame f = std::move(stack.back());
    stack.pop_back();
    const uint64_t code = code_of(f.face, f.level, f.i, f.j);
    auto it = own.find(code);
    if (it != own.end()) f.refs.insert(f.refs.end(), it->second.begin(), it->second.end());
    if (above.count(code)) {
      for (int q = 3; q >= 0; q--)
        stack.push_back({f.face, f.level + 1, (f.i << 1) | (uint32_t)(q >> 1),
                         (f.j << 1) | (uint32_t)(q & 1), f.refs});
      continue;
    }
    if (f.refs.empty()) continue;
    // per polygon: a true hit if any of its cells here is interior
    std::sort(f.refs.begin(), f.refs.end());
    Work w;
    w.face = f.face;
    w.level = f.level;
    w.i = f.i;
    w.j = f.j;
    w.box = inflate(cell_bounds(f.face, f.level, f.i, f.j), bp.margin_deg);
    for (size_t k = 0; k < f.refs.size();) {
      const uint32_t poly = f.refs[k] >> 1;
      bool inside = false;
      for (; k < f.refs.size() && (f.refs[k] >> 1) == poly; k++) inside |= (f.refs[k] & 1u) != 0;
      if (inside)
        w.interior.push_back((int32_t)poly);
      else
        w.bnd.push_back({(int32_t)poly, 0, 0});
    }
    emit(C, w, sink);
  }
}

// ------------------------------------------------------------------- LUT

}  // namespace

struct LutDedup {
  std::unordered_map<std::string, uint32_t> map;
};
LutDedup *lut_dedup_new() { return new LutDedup; }
void lut_dedup_free(LutDedup *d) { delete d; }

static uint64_t encode_refs_impl(const uint32_t *refs, int n, std::vector<uint32_t> &lut,
                                 LutDedup *dedup, bool inline_ok) {
  if (n <= 0) return 0;
  std::vector<uint32_t> r(refs, refs + n);
  std::sort(r.begin(), r.end(), [](uint32_t a, uint32_t b) { return (a >> 1) < (b >> 1); });
  if (inline_ok && n == 1) return ((uint64_t)r[0] << 2) | kTagOne;
  if (inline_ok && n == 2) return ((uint64_t)r[0] << 2) | ((uint64_t)r[1] << 33) | kTagTwo;
  std::vector<uint32_t> list;
  list.reserve(n + 2);
  uint32_t nt = 0;
  for (uint32_t v : r) nt += v & 1u;
  list.push_back(nt);
  for (uint32_t v : r)
    if (v & 1u) list.push_back(v >> 1);
  list.push_back((uint32_t)n - nt);
  for (uint32_t v : r)
    if (!(v & 1u)) list.push_back(v >> 1);
  std::string key((const char *)list.data(), list.size() * sizeof(uint32_t));
  auto it = dedup->map.find(key);
  uint32_t off;
  if (it != dedup->map.end()) {
    off = it->second;
  } else {
    off = (uint32_t)lut.size();
    lut.insert(lut.end(), list.begin(), list.end());
    dedup->map.emplace(std::move(key), off);
  }
  return ((uint64_t)off << 2) | kTagLut;
}

uint64_t encode_refs(const uint32_t *refs, int n, std::vector<uint32_t> &lut, LutDedup *dedup) {
  return encode_refs_impl(refs, n, lut, dedup, true);
}

uint64_t encode_refs_lut(const uint32_t *refs, int n, std::vector<uint32_t> &lut, LutDedup *dedup) {
  return encode_refs_impl(refs, n, lut, dedup, false);
}

// The device keeps every trie entry in 32 bits (1 KiB nodes: half the HBM
// footprint and twice the entries per cache line; the GPU also stages the
// top levels in LDS). An entry fits when its high 32 bits are zero: child
// pointers, lookup-table offsets and single references of polygon ids below
// 2^29. The others -- two inlined references, or a single reference of a
// larger id -- are rewritten as (deduplicated) lookup-table references.
static void narrow_entries(HostIndex &x, LutDedup *dedup) {
  for (size_t k = 256; k < x.nodes.size(); k++) {
    const uint64_t e = x.nodes[k];
    if ((e >> 32) == 0) continue;
    uint32_t refs[2];
    int n = 0;
    refs[n++] = (uint32_t)((e >> 2) & 0x7fffffffu);
    if ((e & kTagMask) == kTagTwo) refs[n++] = (uint32_t)((e >> 33) & 0x7fffffffu);
    x.nodes[k] = encode_refs_lut(refs, n, x.lut, dedup);
  }
}

uint64_t host_lookup(const HostIndex &idx, int face, uint32_t i, uint32_t j) {
  if (face < 0 || face > 5) return 0;
  const FaceRoot &f = idx.faces[face];
  if (f.root < 0) return 0;
  int sh = kMaxLevel - f.plevel;
  if ((i >> sh) != f.pi || (j >> sh) != f.pj) return 0;
  uint64_t node = (uint64_t)f.root;
  for (;;) {
    sh -= 4;
    uint64_t e = idx.nodes[node * 256 + node_slot(i, j, sh)];
    if ((e & kTagMask) != kTagPtr || e == 0) return e;
    node = e >> 2;
  }
}

// Renumber trie nodes breadth-first (roots, then their children, ...) and
// rewrite child pointers accordingly.
static void renumber_breadth_first(HostIndex &x) {
  size_t n_nodes = x.nodes.size() / 256;
  std::vector<uint64_t> order;
  std::vector<int> depth;
  order.reserve(n_nodes);
  for (int f = 0; f < 6; f++)
    if (x.faces[f].root >= 0) {
      order.push_back((uint64_t)x.faces[f].root);
      depth.push_back(0);
    }
  for (size_t q = 0; q < order.size(); q++) {
    const uint64_t *e = &x.nodes[order[q] * 256];
    for (int b = 0; b < 256; b++)
      if ((e[b] & kTagMask) == kTagPtr && e[b] != 0) {
        order.push_back(e[b] >> 2);
        depth.push_back(depth[q] + 1);
      }
  }
  std::vector<uint64_t> newidx(n_nodes, 0);
  for (size_t q = 0; q < order.size(); q++) newidx[order[q]] = q + 1;
  for (size_t o = 1, q = order.size(); o < n_nodes; o++)  // unreachable nodes (none expected) last
    if (newidx[o] == 0) newidx[o] = ++q;
  order.clear();
  order.shrink_to_fit();
  // rewrite the child pointers, then move every node to its new index in
  // place (cycle by cycle, one node of scratch)
  for (size_t o = 1; o < n_nodes; o++) {
    uint64_t *e = &x.nodes[o * 256];
    for (int b = 0; b < 256; b++)
      if ((e[b] & kTagMask) == kTagPtr && e[b] != 0) e[b] = newidx[e[b] >> 2] << 2;
  }
  std::vector<bool> done(n_nodes, false);
  uint64_t buf[256];
  for (size_t s = 1; s < n_nodes; s++) {
    if (done[s] || newidx[s] == s) continue;
    std::memcpy(buf, &x.nodes[s * 256], sizeof buf);
    size_t cur = s;
    do {
      const size_t d = newidx[cur];
      done[cur] = true;
      std::swap_ranges(buf, buf + 256, &x.nodes[d * 256]);
      cur = d;
    } while (cur != s);
  }
  for (int f = 0; f < 6; f++)
    if (x.faces[f].root >= 0) x.faces[f].root = (int32_t)newidx[x.faces[f].root];
  x.n_d0 = x.n_d1 = 0;
  for (int d : depth) {
    x.n_d0 += d == 0;
    x.n_d1 += d == 1;
  }
}

// 30 bits of i and j interleaved (i above j at each level), so that sorting
// by the key lists the cells in quadtree (depth-first) order.
static uint64_t spread30(uint32_t v) {
  uint64_t x = v & 0x3fffffffu;
  x = (x | (x << 16)) & 0x0000ffff0000ffffull;
  x = (x | (x << 8)) & 0x00ff00ff00ff00ffull;
  x = (x | (x << 4)) & 0x0f0f0f0f0f0f0f0full;
  x = (x | (x << 2)) & 0x3333333333333333ull;
  x = (x | (x << 1)) & 0x5555555555555555ull;
  return x;
}

static uint64_t quad_key(uint32_t i, uint32_t j) { return (spread30(i) << 1) | spread30(j); }

// Cells of the super covering, sorted by (face, quadtree key) for the trie
// build.
struct Cell {
  int face, level;
  uint32_t I, J;            // leaf coordinates of the cell's first leaf
  uint64_t key;             // quadtree path of that leaf: bits of I and J interleaved
  const uint32_t *refs;
  const uint32_t *locs;
  uint64_t local_base;      // offset of the cell's sink in the local records
  int n;
};

constexpr int64_t kPrefixGrowth = 8;
constexpr int64_t kPrefixMaxNodes = (4ll << 30) / 2048;  // 4 GiB of nodes

// The cells of each face: range [c0, c1) of the sorted cells, the deepest
// level all of them share (common ancestor, capped by the coarsest cell)
// and the finest cell level.
struct FaceCells {
  size_t c0 = 0, c1 = 0;
  int lc = 0, lmax = 0;
};

static void face_ranges(const std::vector<Cell> &cells, FaceCells fc[6]) {
  size_t c0 = 0;
  for (int face = 0; face < 6; face++) {
    size_t c1 = c0;
    while (c1 < cells.size() && cells[c1].face == face) c1++;
    FaceCells &F = fc[face];
    F.c0 = c0;
    F.c1 = c1;
    int lmin = 30, lmax = 0;
    uint32_t diff = 0;
    for (size_t k = c0; k < c1; k++) {
      lmin = std::min(lmin, cells[k].level);
      lmax = std::max(lmax, cells[k].level);
      diff |= (cells[k].I ^ cells[c0].I) | (cells[k].J ^ cells[c0].J);
    }
    const int common = diff ? 29 - (31 - __builtin_clz(diff)) : 30;
    F.lc = std::min(lmin, common);
    F.lmax = lmax;
    c0 = c1;
  }
}

// Nodes a face's trie needs with prefix level lp: the root, plus per node
// depth d >= 1 the distinct ancestors at level lp + 4d of the cells finer
// than that level. The cells are in quadtree order, so equal ancestors are
// adjacent. `depth1` receives the count at depth 1.
static int64_t count_nodes(const std::vector<Cell> &cells, const FaceCells &F, int lp,
                           int64_t &depth1) {
  int64_t total = 1;
  depth1 = 0;
  for (int d = 1; lp + 4 * d < F.lmax; d++) {
    const int L = lp + 4 * d, s = 2 * (kMaxLevel - L);
    int64_t u = 0;
    uint64_t last = ~0ull;
    for (size_t k = F.c0; k < F.c1; k++)
      if (cells[k].level > L && (cells[k].key >> s) != last) {
        last = cells[k].key >> s;
        u++;
      }
    total += u;
    if (d == 1) depth1 = u;
  }
  return total;
}

// Prefix levels of the faces. Default: the common-ancestor level lowered (by
// at most 3) so that the finest cells end a node level, which keeps the
// most numerous cells from being replicated. The common-ancestor level
// itself moves the two LDS-staged node levels further down the tree, so
// more points end their descent in LDS; it is taken when those levels still
// fit the probe's LDS budget, the trie grows by at most kPrefixGrowth and
// stays within kPrefixMaxNodes.
// Returns the number of trie nodes (node 0 included) the choice needs.
static int64_t choose_prefix(const std::vector<Cell> &cells, const FaceCells fc[6],
                             const BuildParams &bp, int lp[6]) {
  int aligned[6];
  int64_t n_al = 1, n_co = 1, top_co = 0, d1;
  for (int f = 0; f < 6; f++) {
    const FaceCells &F = fc[f];
    aligned[f] = F.lc - ((4 - (F.lmax - F.lc) % 4) % 4);
    if (aligned[f] < 0) aligned[f] = F.lc;
    lp[f] = bp.prefix_level >= 0 ? std::min(bp.prefix_level, F.lc) : aligned[f];
    if (F.c1 == F.c0) continue;
    n_al += count_nodes(cells, F, lp[f], d1);
    if (bp.prefix_level < 0) {
      n_co += count_nodes(cells, F, F.lc, d1);
      top_co += 1 + d1;
    }
  }
  if (bp.prefix_level < 0 && top_co <= kLdsTrieNodes && n_co <= kPrefixGrowth * n_al &&
      n_co <= kPrefixMaxNodes) {
    for (int f = 0; f < 6; f++) lp[f] = fc[f].lc;
    return n_co;
  }
  return n_al;
}

// ------------------------------------------------------------- training
//
// Section III-D: when a training point hits an expensive cell (one whose
// reference list has a candidate), that cell is replaced by its four
// children, each classified against the cell's references (a polygon
// interior to the parent stays interior; a candidate polygon becomes
// interior, candidate or absent per child), and the index is updated. This
// is repeated, one split per hit, over the training points in their order
// until the memory budget is used up. The image's size is tracked as the
// training goes: the trie nodes (with the faces' prefix levels fixed before
// training) and an upper bound of the lookup-table words each cell needs.

// Leaf cell (face, i, j) of a point, by the projection of cellid.hpp (host
// trigonometry). Training only chooses which cells to split, so the host's
// rounding does not matter for the join's results.
static bool host_leaf(double lat, double lng, int &face, uint32_t &i, uint32_t &j) {
  if (!(std::fabs(lat) <= 90.0 && std::fabs(lng) <= 180.0)) return false;
  const double phi = lat / kDeg, lam = lng / kDeg;
  const double c[3] = {std::cos(phi) * std::cos(lam), std::cos(phi) * std::sin(lam), std::sin(phi)};
  const double ax = std::fabs(c[0]), ay = std::fabs(c[1]), az = std::fabs(c[2]);
  const int a = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
  const double m = std::fabs(c[a]);
  face = a + (c[a] < 0 ? 3 : 0);
  auto coord = [](double w) {
    const double v = std::floor(kTwo30 * st_from_uv(w));
    return (uint32_t)std::min(std::max(v, 0.0), kTwo30 - 1.0);
  };
  i = coord(c[(a + 1) % 3] / m);
  j = coord(c[(a + 2) % 3] / m);
  return true;
}

// Unique key of a cell (coordinates at its level): face, quadtree path and
// a marker bit, laid out like a cell id.
static uint64_t cell_code(int face, int level, uint32_t i, uint32_t j) {
  const int sh = 2 * (kMaxLevel - level);
  return ((uint64_t)face << 61) | (quad_key(i, j) << (sh + 1)) | (1ull << sh);
}


// Lookup-table words a cell needs at most (deduplication can only save):
// with 32-bit trie entries, a cell with two references (or a reference id
// of 2^29 or more) has a list too. `top` is unused.
static int64_t cell_lut_words(const Cell &c, const std::vector<uint32_t> &local, bool exact,
                              bool top) {
  (void)top;  // `exact`: the cell's candidates carry cell-local records
  int nt = 0, nc = 0;
  int64_t rec = 0;
  for (int r = 0; r < c.n; r++) {
    if (c.refs[r] & 1u) {
      nt++;
    } else {
      nc++;
      if (exact) {
        const uint32_t *w = &local[c.local_base + c.locs[r]];
        rec += 2 + 8 * (int64_t)w[0] + 2 * (int64_t)(w[1] & 0x7fffffffu);
      }
    }
  }
  if (exact && nc > 0) return 2 + nt + 2 * (int64_t)nc + rec;
  return c.n >= 2 || (c.n == 1 && (c.refs[0] >> 1) >= (1u << 29)) ? 2 + c.n : 0;
}

// Node level of a cell at level l under prefix level lp.
static int node_depth(int l, int lp) { return l <= lp ? 0 : (l - lp - 1) / 4; }

struct Trainer {
  Ctx &C;
  const Prep &P;
  std::vector<Cell> &cells;
  std::vector<uint32_t> &local;
  std::deque<std::vector<uint32_t>> &store;  // refs and locs of cells made by splits
  std::unordered_map<uint64_t, size_t> where;  // cell code -> index in cells
  std::unordered_set<uint64_t> nodes;          // (face, ancestor at lp + 4d) of every node
  int64_t top_nodes = 0;                       // nodes at depths 0 and 1
  int lp[6];
  int lcap[6];  // finest level a face's node alignment allows
  uint32_t levels = 0;  // bit l: some cell has level l

  Trainer(Ctx &c, const Prep &p, std::vector<Cell> &cs, std::vector<uint32_t> &lc,
          std::deque<std::vector<uint32_t>> &st)
      : C(c), P(p), cells(cs), local(lc), store(st) {}

  void add_nodes(const Cell &c) {
    const int l = c.level, f = c.face;
    for (int d = 0; d <= node_depth(l, lp[f]); d++) {
      const int L = lp[f] + 4 * d;
      const int sh = kMaxLevel - L;
      if (nodes.insert(cell_code(f, L, c.I >> sh, c.J >> sh)).second && d <= 1) top_nodes++;
    }
  }

  // Index of the cell containing leaf (face, i, j), or SIZE_MAX.
  size_t find(int face, uint32_t i, uint32_t j) const {
    for (int l = kMaxLevel; l >= 0; l--) {
      if (!((levels >> l) & 1u)) continue;
      const int sh = kMaxLevel - l;
      auto it = where.find(cell_code(face, l, i >> sh, j >> sh));
      if (it != where.end()) return it->second;
    }
    return SIZE_MAX;
  }

  // Children of cell k (their cells appended to `kids`, records to local).
  void split(size_t k, std::vector<Cell> &kids) {
    const Cell c = cells[k];
    const int sh = kMaxLevel - c.level;
    Work w;
    w.face = c.face;
    w.level = c.level;
    w.i = c.I >> sh;
    w.j = c.J >> sh;
    w.box = inflate(cell_bounds(w.face, w.level, w.i, w.j), C.bp.margin_deg);
    for (int r = 0; r < c.n; r++) {
      const int32_t p = (int32_t)(c.refs[r] >> 1);
      if (c.refs[r] & 1u) {
        w.interior.push_back(p);
      } else {
        const int32_t off = (int32_t)w.edges.size();
        for (int e = P.e_off[p]; e < P.e_off[p + 1]; e++) w.edges.push_back(e);
        w.bnd.push_back({p, off, P.e_off[p + 1] - P.e_off[p]});
      }
    }
    Sink tmp;
    Work ch;
    for (int q = 0; q < 4; q++) {
      make_child(C, w, q, ch);
      if (ch.bnd.empty() && ch.interior.empty()) continue;  // outside every polygon
      emit(C, ch, tmp);
    }
    const uint64_t base = local.size();
    local.insert(local.end(), tmp.local.begin(), tmp.local.end());
    for (const CellOut &o : tmp.cells) {
      store.emplace_back(tmp.refs.begin() + o.ref_off, tmp.refs.begin() + o.ref_off + o.ref_cnt);
      const uint32_t *refs = store.back().data();
      std::vector<uint32_t> locs(tmp.locs.begin() + o.ref_off,
                                 tmp.locs.begin() + o.ref_off + o.ref_cnt);
      for (uint32_t &v : locs)
        if (v != UINT32_MAX) v = (uint32_t)(base + v);
      store.push_back(std::move(locs));
      const int s2 = kMaxLevel - o.level;
      kids.push_back({o.face, o.level, o.i << s2, o.j << s2, quad_key(o.i << s2, o.j << s2), refs,
                      store.back().data(), 0, o.ref_cnt});
    }
  }
};

// `store` receives the reference arrays of the cells the splits make (the
// cells point into it, so it must outlive the trie build).
static void train_index(Ctx &C, const Prep &P, std::vector<Cell> &cells,
                        std::vector<uint32_t> &local, std::deque<std::vector<uint32_t>> &store,
                        const int lp[6], int64_t fixed_bytes, HostIndex &out) {
  const BuildParams &bp = C.bp;
  const bool exact = bp.mode == ACT_EXACT && bp.geometry == ACT_GEOM_PLANE;  // with records
  Trainer T(C, P, cells, local, store);
  int64_t lut_words = 10;  // the device copy's padding
  for (int f = 0; f < 6; f++) {
    T.lp[f] = lp[f];
    T.lcap[f] = std::min(bp.train_max_level, lp[f] + 4 * ((kMaxLevel - lp[f]) / 4));
  }
  for (size_t k = 0; k < cells.size(); k++) {
    const Cell &c = cells[k];
    T.where[cell_code(c.face, c.level, c.I >> (kMaxLevel - c.level), c.J >> (kMaxLevel - c.level))] = k;
    T.levels |= 1u << c.level;
    T.add_nodes(c);
    lut_words += cell_lut_words(c, local, exact, node_depth(c.level, T.lp[c.face]) <= 1);
  }
  auto bytes = [&](int64_t n_nodes, int64_t top, int64_t words) {
    (void)top;
    return fixed_bytes + (n_nodes + 1) * 1024 + 4 * words;
  };
  if (bp.memory_budget > 0 &&
      bytes((int64_t)T.nodes.size(), T.top_nodes, lut_words) > bp.memory_budget)
    return;  // the untrained index already uses the budget
  std::vector<Cell> kids;
  int64_t used = 0;
  for (; used < bp.n_train; used++) {
    int face;
    uint32_t i, j;
    if (!host_leaf(bp.train_points[2 * used], bp.train_points[2 * used + 1], face, i, j)) continue;
    const size_t k = T.find(face, i, j);
    if (k == SIZE_MAX) continue;  // a false hit
    const Cell c = cells[k];
    bool expensive = false;
    for (int r = 0; r < c.n; r++) expensive |= !(c.refs[r] & 1u);
    if (!expensive || c.level >= T.lcap[face]) continue;
    kids.clear();
    T.split(k, kids);
    // what the split adds: a new node when the children start a node level,
    // and the children's lists in place of the parent's
    const int lpf = T.lp[face];
    int64_t words = lut_words - cell_lut_words(c, local, exact, node_depth(c.level, lpf) <= 1);
    for (const Cell &q : kids)
      words += cell_lut_words(q, local, exact, node_depth(q.level, lpf) <= 1);
    const bool new_node = node_depth(c.level + 1, T.lp[face]) > node_depth(c.level, T.lp[face]);
    const uint64_t nkey = cell_code(face, c.level, c.I >> (kMaxLevel - c.level),
                                    c.J >> (kMaxLevel - c.level));
    const bool adds = new_node && !T.nodes.count(nkey);
    const int64_t top = T.top_nodes + (adds && node_depth(c.level + 1, T.lp[face]) <= 1);
    if (bp.memory_budget > 0 &&
        bytes((int64_t)T.nodes.size() + (adds ? 1 : 0), top, words) > bp.memory_budget)
      break;  // the budget is used up
    if (adds) {
      T.nodes.insert(nkey);
      T.top_nodes = top;
    }
    lut_words = words;
    T.where.erase(cell_code(face, c.level, c.I >> (kMaxLevel - c.level), c.J >> (kMaxLevel - c.level)));
    cells[k].n = -1;  // replaced by its children
    for (const Cell &q : kids) {
      T.where[cell_code(q.face, q.level, q.I >> (kMaxLevel - q.level), q.J >> (kMaxLevel - q.level))] =
          cells.size();
      T.levels |= 1u << q.level;
      cells.push_back(q);
    }
    out.train_splits++;
  }
  out.train_points_used = used;
  std::vector<Cell> live;  // without the cells that were split
  live.reserve(cells.size());
  for (const Cell &c : cells)
    if (c.n >= 0) live.push_back(c);
  cells.swap(live);
}

// Builds the faces' tries and lookup table from the sorted cells into
// out.nodes / out.lut / out.faces (and the trie statistics), with prefix
// level lp[face].
static int build_tries(const std::vector<Cell> &cells, const FaceCells fc[6], const int lp_face[6],
                       int64_t n_nodes, const std::vector<uint32_t> &local, HostIndex &out,
                       const BuildParams &bp, std::string &err) {
  out.nodes.clear();
  out.lut.clear();
  for (int f = 0; f < 6; f++) out.faces[f] = FaceRoot();
  out.max_depth = out.max_refs = out.max_cell_level = 0;
  out.n_cells_interior_only = 0;
  out.local_words = 0;
  out.nodes.reserve(256 * (size_t)n_nodes);
  out.nodes.assign(256, 0);  // node 0 reserved
  LutDedup dedup;
  for (int face = 0; face < 6; face++) {
    const size_t c0 = fc[face].c0, c1 = fc[face].c1;
    if (c1 == c0) continue;
    // node levels Lp+1..Lp+4, Lp+5..Lp+8, ...
    const int lp = lp_face[face];
    if (lp + 4 * ((fc[face].lmax - lp + 3) / 4) > kMaxLevel) {
      err = "cells on one face span too wide a range for the trie's level alignment";
      return ACT_E_RANGE;
    }
    FaceRoot &F = out.faces[face];
    F.plevel = lp;
    F.pi = cells[c0].I >> (kMaxLevel - lp);
    F.pj = cells[c0].J >> (kMaxLevel - lp);
    F.root = (int32_t)(out.nodes.size() / 256);
    out.nodes.resize(out.nodes.size() + 256, 0);
    for (size_t k = c0; k < c1; k++) {
      const Cell &c = cells[k];
      int l = c.level;
      int kd = l <= lp ? 0 : (l - lp - 1) / 4;  // node level holding the cell
      uint64_t node = (uint64_t)F.root;
      for (int d = 0; d < kd; d++) {
        uint64_t slot = node * 256 + node_slot(c.I, c.J, kMaxLevel - lp - 4 * (d + 1));
        uint64_t e = out.nodes[slot];
        if (e == 0) {
          uint64_t nn = out.nodes.size() / 256;
          out.nodes[slot] = nn << 2;
          out.nodes.resize(out.nodes.size() + 256, 0);
          node = nn;
        } else if ((e & kTagMask) == kTagPtr) {
          node = e >> 2;
        } else {
          err = "internal: overlapping cells in the super covering";
          return ACT_E_POLY;
        }
      }
      // denormalise: the cell covers a 2^k x 2^k block of the node's 16 x 16
      // (i nibble, j nibble) entries, k = levels between the cell and the
      // node's last level
      const int sh = kMaxLevel - lp - 4 * (kd + 1);
      const uint32_t ni = (c.I >> sh) & 15u, nj = (c.J >> sh) & 15u;
      const uint32_t span = 1u << (lp + 4 * (kd + 1) - l);
      bool has_cand = false;
      for (int r = 0; r < c.n; r++) has_cand |= !(c.refs[r] & 1u);
      uint64_t entry;
      if (has_cand && bp.mode == ACT_EXACT && bp.geometry == ACT_GEOM_PLANE) {
        // candidate cell: lookup-table list, the candidates' record offsets,
        // then the records themselves, so that one contiguous read serves a
        // pending point
        std::vector<uint32_t> tru, cand, locs;
        for (int r = 0; r < c.n; r++) {
          if (c.refs[r] & 1u) {
            tru.push_back(c.refs[r] >> 1);
          } else {
            cand.push_back(c.refs[r] >> 1);
            locs.push_back((uint32_t)(c.local_base + c.locs[r]));
          }
        }
        entry = ((uint64_t)out.lut.size() << 2) | kTagLut;
        out.lut.push_back((uint32_t)tru.size());
        out.lut.insert(out.lut.end(), tru.begin(), tru.end());
        out.lut.push_back((uint32_t)cand.size());
        out.lut.insert(out.lut.end(), cand.begin(), cand.end());
        const size_t at = out.lut.size();
        out.lut.resize(at + locs.size());
        for (size_t r = 0; r < locs.size(); r++) {
          const uint32_t *rec = &local[locs[r]];
          const size_t len = 2 + 8 * (size_t)rec[0] + 2 * (size_t)(rec[1] & 0x7fffffffu);
          out.lut[at + r] = (uint32_t)out.lut.size();
          out.lut.insert(out.lut.end(), rec, rec + len);
          out.local_words += (int64_t)len;
        }
      } else {
        entry = encode_refs(c.refs, c.n, out.lut, &dedup);
      }
      if (out.lut.size() >= (1ull << 31)) {
        err = "lookup table exceeds 2^31 words";
        return ACT_E_RANGE;
      }
      for (uint32_t a = 0; a < span; a++)
        for (uint32_t b = 0; b < span; b++) {
          uint64_t slot = node * 256 + (((ni + a) << 4) | (nj + b));
          if (out.nodes[slot] != 0) {
            err = "internal: overlapping cells in the super covering";
            return ACT_E_POLY;
          }
          out.nodes[slot] = entry;
        }
      F.depth = std::max(F.depth, kd + 1);
      out.max_depth = std::max(out.max_depth, kd + 1);
      out.max_refs = std::max(out.max_refs, c.n);
      out.max_cell_level = std::max(out.max_cell_level, l);
      bool all_true = true;
      for (int r = 0; r < c.n; r++) all_true &= (c.refs[r] & 1u) != 0;
      out.n_cells_interior_only += all_true;
    }
  }
  renumber_breadth_first(out);
  narrow_entries(out, &dedup);
  if (out.lut.size() >= (1ull << 30)) {
    err = "lookup table exceeds 2^30 words";
    return ACT_E_RANGE;
  }
  if (out.nodes.size() / 256 >= (1ull << 30)) {  // pointer entries carry 30-bit node indices
    err = "trie exceeds 2^30 nodes";
    return ACT_E_RANGE;
  }
  return ACT_OK;
}

int64_t image_fixed_bytes(int64_t n_polys, int64_t n_edges) {
  auto up = [](int64_t b) { return std::max<int64_t>(b, 16); };  // each upload is at least 16 B
  return up(4 * (n_polys + 1)) + up(16 * n_polys) + up(4 * n_polys) + up(16 * n_edges) +
         up(32 * n_edges) + up(361 * 16) + up(6 * 16) + up(64);
}

int64_t image_bytes(const HostIndex &h) {
  return image_fixed_bytes(h.n_polys, (int64_t)h.edges64.size() / 4) +
         std::max<int64_t>(16, (int64_t)h.nodes.size() * 4) + 4 * ((int64_t)h.lut.size() + 10) +
         (h.geometry == ACT_GEOM_SPHERE ? std::max<int64_t>(16, 8 * (int64_t)h.normals.size())
                                        : 0);
}

// Largest distance, in latitude at equal longitude, between the great-circle
// arc from (lat_a, lng_a) to (lat_b, lng_b) and the straight chord between
// them in the lat/lng plane, sampled at 31 interior longitudes (the distance is a
// smooth bump that vanishes at both ends; the caller pads it). The arc's
// latitude at longitude l follows from the plane through both endpoints:
// tan(lat) = (tan(lat_a) sin(lng_b - l) + tan(lat_b) sin(l - lng_a)) /
// sin(lng_b - lng_a). Edges along a meridian coincide with their chord.
static double arc_chord_deviation(double lat_a, double lng_a, double lat_b, double lng_b) {
  if (lng_a == lng_b) return 0.0;
  const double ta = std::tan(lat_a / kDeg), tb = std::tan(lat_b / kDeg);
  const double s = std::sin((lng_b - lng_a) / kDeg);
  double dev = 0;
  for (int k = 1; k < 32; k++) {
    const double f = k / 32.0, l = lng_a + f * (lng_b - lng_a);
    const double t = (ta * std::sin((lng_b - l) / kDeg) + tb * std::sin((l - lng_a) / kDeg)) / s;
    const double lat_arc = std::atan(t) * kDeg;
    dev = std::max(dev, std::fabs(lat_arc - (lat_a + f * (lat_b - lat_a))));
  }
  return dev;
}

// ------------------------------------------------------------ index files

namespace {

constexpr char kFileMagic[8] = {'A', 'C', 'T', 'I', 'D', 'X', '0', '1'};
constexpr uint32_t kFileVersion = 3;  // 2: 32-bit trie entries; 3: geometry

// Running digest of the bytes written or read (FNV-style mixing).
struct Digest {
  uint64_t d = 0xcbf29ce484222325ull;
  void mix(const void *p, size_t n) {
    const uint8_t *b = (const uint8_t *)p;
    for (size_t k = 0; k < n; k++) d = (d ^ b[k]) * 0x100000001b3ull;
  }
};

struct Writer {
  FILE *f;
  Digest dg;
  bool ok = true;
  void raw(const void *p, size_t n) {
    if (n && std::fwrite(p, 1, n, f) != n) ok = false;
    dg.mix(p, n);
  }
  template <typename T> void val(const T &v) { raw(&v, sizeof v); }
  template <typename T> void vec(const std::vector<T> &v) {
    const uint64_t n = v.size();
    val(n);
    raw(v.data(), n * sizeof(T));
  }
};

struct Reader {
  FILE *f;
  Digest dg;
  bool ok = true;
  uint64_t left;  // bytes of the file not read yet
  void raw(void *p, size_t n) {
    if (!ok || n > left || (n && std::fread(p, 1, n, f) != n)) {
      ok = false;
      return;
    }
    left -= n;
    dg.mix(p, n);
  }
  template <typename T> void val(T &v) { raw(&v, sizeof v); }
  template <typename T> void vec(std::vector<T> &v) {
    uint64_t n = 0;
    val(n);
    if (!ok || n > left / sizeof(T)) {
      ok = false;
      return;
    }
    v.resize(n);
    raw(v.data(), n * sizeof(T));
  }
};

template <typename IO, typename H>
void scalars(IO &io, H &h) {
  io.val(h.mode);
  io.val(h.precision_m);
  io.val(h.max_level);
  io.val(h.n_polys);
  for (int f = 0; f < 6; f++) {
    io.val(h.faces[f].root);
    io.val(h.faces[f].plevel);
    io.val(h.faces[f].pi);
    io.val(h.faces[f].pj);
    io.val(h.faces[f].depth);
  }
  io.val(h.local_words);
  io.val(h.n_cells);
  io.val(h.n_cells_interior_only);
  io.val(h.max_depth);
  io.val(h.max_refs);
  io.val(h.max_cell_level);
  io.val(h.n_d0);
  io.val(h.n_d1);
  io.val(h.build_seconds);
  io.val(h.train_splits);
  io.val(h.train_points_used);
  io.val(h.geometry);
  io.val(h.margin_deg);
}

template <typename IO, typename H>
void arrays(IO &io, H &h) {
  io.vec(h.nodes);
  io.vec(h.lut);
  io.vec(h.poly_edge_off);
  io.vec(h.poly_origin);
  io.vec(h.poly_m);
  io.vec(h.edges32);
  io.vec(h.edges64);
  io.vec(h.normals);
}

}  // namespace

// Every reference the probe follows stays inside the image: child pointers
// name existing nodes, lookup-table lists and the cell-local records they
// point to lie inside the table, polygon ids are below n_polys, and the
// faces' roots and prefix levels are valid.
static bool image_consistent(const HostIndex &h) {
  const uint64_t n_nodes = h.nodes.size() / 256, n_lut = h.lut.size();
  const uint32_t np = (uint32_t)h.n_polys;
  if (n_nodes == 0 || (uint64_t)h.n_d0 + (uint64_t)h.n_d1 >= n_nodes || h.n_d0 < 0 || h.n_d1 < 0)
    return false;
  for (int f = 0; f < 6; f++) {
    const FaceRoot &F = h.faces[f];
    if (F.root != -1 && (F.root <= 0 || (uint64_t)F.root >= n_nodes)) return false;
    if (F.plevel < 0 || F.plevel > kMaxLevel) return false;
  }
  const bool exact = h.mode == ACT_EXACT && h.geometry == ACT_GEOM_PLANE;  // lists with records
  if (h.geometry == ACT_GEOM_SPHERE && h.normals.size() != 3 * (h.edges64.size() / 4)) return false;
  uint64_t last_ok = UINT64_MAX;
  for (uint64_t k = 256; k < h.nodes.size(); k++) {
    const uint64_t e = h.nodes[k];
    if (e == 0) continue;
    if (e >> 32) return false;  // the device keeps 32-bit entries
    switch (e & kTagMask) {
      case kTagPtr:
        if ((e >> 2) == 0 || (e >> 2) >= n_nodes) return false;
        break;
      case kTagTwo:
        if ((((e >> 33) & 0x7fffffffu) >> 1) >= np) return false;
        [[fallthrough]];
      case kTagOne:
        if ((((e >> 2) & 0x7fffffffu) >> 1) >= np) return false;
        break;
      default: {
        const uint64_t off = e >> 2;
        if (off == last_ok) break;
        if (off + 2 > n_lut) return false;
        const uint64_t nt = h.lut[off];
        if (off + 2 + nt > n_lut) return false;
        const uint64_t nc = h.lut[off + 1 + nt];
        const uint64_t end = off + 2 + nt + nc + (exact && nc ? nc : 0);
        if (end > n_lut) return false;
        for (uint64_t r = 0; r < nt; r++)
          if (h.lut[off + 1 + r] >= np) return false;
        for (uint64_t r = 0; r < nc; r++) {
          if (h.lut[off + 2 + nt + r] >= np) return false;
          if (!exact) continue;
          const uint64_t rec = h.lut[off + 2 + nt + nc + r];
          if (rec + 2 > n_lut) return false;
          const uint64_t len = 2 + 8 * (uint64_t)h.lut[rec] + 2 * (uint64_t)(h.lut[rec + 1] & 0x7fffffffu);
          if (rec + len > n_lut) return false;
        }
        last_ok = off;
      }
    }
  }
  for (uint64_t k = 0; k < (uint64_t)h.n_polys; k++)
    if (h.poly_edge_off[k] > h.poly_edge_off[k + 1]) return false;
  return h.poly_edge_off.empty() || (h.poly_edge_off[0] == 0 &&
         (uint64_t)h.poly_edge_off[h.n_polys] == h.edges64.size() / 4);
}

int save_host_index(const HostIndex &h, const void *extra, uint32_t extra_bytes, const char *path,
                    std::string &err) {
  FILE *f = std::fopen(path, "wb");
  if (!f) {
    err = std::string("cannot open ") + path + " for writing";
    return ACT_E_ARG;
  }
  Writer w{f};
  w.raw(kFileMagic, sizeof kFileMagic);
  w.val(kFileVersion);
  w.val(extra_bytes);
  scalars(w, h);
  arrays(w, h);
  w.raw(extra, extra_bytes);
  const uint64_t d = w.dg.d;
  w.val(d);
  const bool ok = w.ok && std::fclose(f) == 0;
  if (!ok) {
    err = std::string("writing ") + path + " failed";
    return ACT_E_ARG;
  }
  return ACT_OK;
}

int load_host_index(const char *path, HostIndex &h, void *extra, uint32_t extra_bytes,
                    std::string &err) {
  FILE *f = std::fopen(path, "rb");
  if (!f) {
    err = std::string("cannot open ") + path;
    return ACT_E_ARG;
  }
  std::fseek(f, 0, SEEK_END);
  const long size = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  Reader r{f};
  r.left = size > 0 ? (uint64_t)size : 0;
  char magic[8];
  uint32_t version = 0, xb = 0;
  r.raw(magic, sizeof magic);
  r.val(version);
  r.val(xb);
  if (!r.ok || std::memcmp(magic, kFileMagic, 8) != 0 || version != kFileVersion ||
      xb != extra_bytes) {
    std::fclose(f);
    err = std::string(path) + " is not an index file of this version";
    return ACT_E_ARG;
  }
  h = HostIndex();
  scalars(r, h);
  arrays(r, h);
  r.raw(extra, extra_bytes);
  const uint64_t want = r.dg.d;
  uint64_t got = 0;
  r.val(got);
  std::fclose(f);
  const bool shape_ok = h.n_polys >= 0 && h.poly_edge_off.size() == (size_t)h.n_polys + 1 &&
                        h.nodes.size() % 256 == 0 && h.poly_origin.size() == 2 * (size_t)h.n_polys &&
                        h.poly_m.size() == (size_t)h.n_polys && h.edges64.size() % 4 == 0 &&
                        h.edges32.size() == h.edges64.size() &&
                        (h.mode == ACT_EXACT || h.mode == ACT_APPROX) &&
                        (h.geometry == ACT_GEOM_PLANE || h.geometry == ACT_GEOM_SPHERE);
  if (!r.ok || got != want || r.left != 0 || !shape_ok || !image_consistent(h)) {
    h = HostIndex();
    err = std::string(path) + ": truncated or corrupt index file";
    return ACT_E_ARG;
  }
  return ACT_OK;
}

// The physical index (Section III-C) from the emitted cells: gathered,
// sorted, trained (exact mode), laid out as tries and lookup table.
static int finish_build(Ctx &C, const Prep &P, const BuildParams &bp, std::vector<Sink> &sinks,
                        HostIndex &out, std::string &err,
                        std::chrono::steady_clock::time_point t0, int32_t n_polys) {
  // gather cells; a cell is addressed by its first leaf (I, J) = (i, j)
  // shifted to level 30
  std::vector<Cell> cells;
  std::vector<uint32_t> local;  // all sinks' records, embedded in the lookup table below
  auto gather = [&](const Sink &s) {
    const uint64_t base = local.size();
    local.insert(local.end(), s.local.begin(), s.local.end());
    for (const CellOut &c : s.cells)
      cells.push_back({c.face, c.level, c.i << (kMaxLevel - c.level), c.j << (kMaxLevel - c.level),
                       quad_key(c.i << (kMaxLevel - c.level), c.j << (kMaxLevel - c.level)),
                       &s.refs[c.ref_off], &s.locs[c.ref_off], base, c.ref_cnt});
  };
  for (const Sink &s : sinks) gather(s);
  if (local.size() >= (1ull << 32)) {
    err = "cell-local refinement records exceed 2^32 words";
    return ACT_E_RANGE;
  }
  auto by_key = [](const Cell &a, const Cell &b) {
    return a.face != b.face ? a.face < b.face : a.key < b.key;
  };
  std::sort(cells.begin(), cells.end(), by_key);
  // ------------------------------------------------------------- tries
  FaceCells fc[6];
  face_ranges(cells, fc);
  int lp[6];
  int64_t n_nodes = choose_prefix(cells, fc, bp, lp);
  std::deque<std::vector<uint32_t>> trained;  // reference arrays of cells made by training
  if (bp.mode == ACT_EXACT && bp.n_train > 0) {
    // training keeps the faces' prefix levels: the trie grows only below them
    train_index(C, P, cells, local, trained, lp,
                image_fixed_bytes(n_polys, (int64_t)(P.ex.size() / 4)), out);
    if (local.size() >= (1ull << 32)) {
      err = "cell-local refinement records exceed 2^32 words";
      return ACT_E_RANGE;
    }
    std::sort(cells.begin(), cells.end(), by_key);
    face_ranges(cells, fc);
    n_nodes = 1;
    for (int f = 0; f < 6; f++) {
      int64_t d1;
      if (fc[f].c1 > fc[f].c0) n_nodes += count_nodes(cells, fc[f], lp[f], d1);
    }
  }
  out.n_cells = (int64_t)cells.size();
  const int rc = build_tries(cells, fc, lp, n_nodes, local, out, bp, err);
  if (rc) return rc;
  out.build_seconds =
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return ACT_OK;
}

int build_host_index(const double *verts, const int64_t *ring_off, const int32_t *poly_ring_off,
                     int32_t n_polys, const BuildParams &bp, HostIndex &out, std::string &err) {
  auto t0 = std::chrono::steady_clock::now();
  if (n_polys < 0 || n_polys > (1 << 30)) {
    err = "n_polys must be in 0 .. 2^30";
    return ACT_E_POLY;
  }
  // ------------------------------------------------ validate and prepare
  Prep P;
  P.n_polys = n_polys;
  P.e_off.assign(n_polys + 1, 0);
  P.bbox.resize(n_polys);
  out = HostIndex();
  out.mode = bp.mode;
  out.precision_m = bp.precision_m;
  out.max_level = bp.max_level;
  out.n_polys = n_polys;
  out.poly_edge_off.assign(n_polys + 1, 0);
  out.poly_origin.resize(2 * (size_t)n_polys);
  out.poly_m.resize(n_polys);
  if (poly_ring_off[0] != 0) {
    err = "poly_ring_off[0] must be 0";
    return ACT_E_POLY;
  }
  for (int p = 0; p < n_polys; p++) {
    int r0 = poly_ring_off[p], r1 = poly_ring_off[p + 1];
    if (r1 <= r0) {
      err = "polygon " + std::to_string(p) + " has no ring";
      return ACT_E_POLY;
    }
    Box bb{INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int r = r0; r < r1; r++) {
      int64_t k0 = ring_off[r], k1 = ring_off[r + 1];
      if (k1 < k0) {
        err = "ring offsets must be non-decreasing";
        return ACT_E_POLY;
      }
      std::vector<double> ring;  // x y pairs after dropping duplicates
      for (int64_t k = k0; k < k1; k++) {
        double lat = verts[2 * k], lng = verts[2 * k + 1];
        if (!std::isfinite(lat) || !std::isfinite(lng) || std::fabs(lat) > 90 ||
            std::fabs(lng) > 180) {
          err = "polygon " + std::to_string(p) + ": vertex out of range or not finite";
          return ACT_E_POLY;
        }
        size_t m = ring.size();
        if (m >= 2 && ring[m - 2] == lng && ring[m - 1] == lat) continue;
        ring.push_back(lng);
        ring.push_back(lat);
      }
      while (ring.size() >= 4 && ring[0] == ring[ring.size() - 2] && ring[1] == ring.back()) {
        ring.pop_back();
        ring.pop_back();
      }
      size_t m = ring.size() / 2;
      if (m < 3) {
        err = "polygon " + std::to_string(p) + ": ring with fewer than 3 distinct vertices";
        return ACT_E_POLY;
      }
      for (size_t k = 0; k < m; k++) {
        size_t kn = (k + 1) % m;
        P.ex.insert(P.ex.end(), {ring[2 * k], ring[2 * k + 1], ring[2 * kn], ring[2 * kn + 1]});
        bb.lng0 = std::min(bb.lng0, ring[2 * k]);
        bb.lng1 = std::max(bb.lng1, ring[2 * k]);
        bb.lat0 = std::min(bb.lat0, ring[2 * k + 1]);
        bb.lat1 = std::max(bb.lat1, ring[2 * k + 1]);
      }
    }
    P.e_off[p + 1] = (int32_t)(P.ex.size() / 4);
    P.bbox[p] = bb;
  }
  if (P.ex.size() / 4 > (size_t)INT32_MAX) {
    err = "too many edges";
    return ACT_E_POLY;
  }
  // ------------------------------------------------------- polygon store
  size_t n_edges = P.ex.size() / 4;
  out.poly_edge_off = P.e_off;
  out.edges64 = P.ex;
  out.edges32.resize(4 * n_edges);
  for (int p = 0; p < n_polys; p++) {
    double ox = 0.5 * (P.bbox[p].lng0 + P.bbox[p].lng1);
    double oy = 0.5 * (P.bbox[p].lat0 + P.bbox[p].lat1);
    out.poly_origin[2 * p] = ox;
    out.poly_origin[2 * p + 1] = oy;
    // fp32 copy translated by the origin and oriented upward (lower
    // endpoint first); the fp64 copy keeps the input orientation
    float m = 0;
    for (int e = P.e_off[p]; e < P.e_off[p + 1]; e++) {
      const double *q = &P.ex[4 * (size_t)e];
      const bool flip = q[1] > q[3];
      const double src[4] = {flip ? q[2] : q[0], flip ? q[3] : q[1], flip ? q[0] : q[2],
                             flip ? q[1] : q[3]};
      for (int c = 0; c < 4; c++) {
        float v = (float)(src[c] - ((c & 1) ? oy : ox));
        out.edges32[4 * (size_t)e + c] = v;
        m = std::max(m, std::fabs(v));
      }
    }
    out.poly_m[p] = m;
  }
  // ------------------------------------------------------ spherical edges
  BuildParams bpx = bp;
  out.geometry = bp.geometry;
  if (bp.geometry == ACT_GEOM_SPHERE) {
    // great-circle normals, and the cell margin widened by the largest
    // distance (in latitude, at equal longitude) between an edge's arc and
    // its chord, so that chord-based classification holds for the arcs
    out.normals.resize(3 * n_edges);
    double dev = 0;
    for (size_t e = 0; e < n_edges; e++) {
      const double *q = &P.ex[4 * e];  // ax ay bx by = lng lat lng lat
      double a[3], b[3];
      const double ca = std::cos(q[1] / kDeg), cb = std::cos(q[3] / kDeg);
      a[0] = ca * std::cos(q[0] / kDeg);
      a[1] = ca * std::sin(q[0] / kDeg);
      a[2] = std::sin(q[1] / kDeg);
      b[0] = cb * std::cos(q[2] / kDeg);
      b[1] = cb * std::sin(q[2] / kDeg);
      b[2] = std::sin(q[3] / kDeg);
      // (b + a) x (b - a) = 2 (a x b): b - a of nearby endpoints is exact,
      // so the normal keeps its relative precision (a x b would cancel)
      const double s0 = b[0] + a[0], s1 = b[1] + a[1], s2 = b[2] + a[2];
      const double d0 = b[0] - a[0], d1 = b[1] - a[1], d2 = b[2] - a[2];
      out.normals[3 * e] = s1 * d2 - s2 * d1;
      out.normals[3 * e + 1] = s2 * d0 - s0 * d2;
      out.normals[3 * e + 2] = s0 * d1 - s1 * d0;
      dev = std::max(dev, arc_chord_deviation(q[1], q[0], q[3], q[2]));
    }
    bpx.margin_deg = bp.margin_deg + 1.25 * dev + 1e-12;
  }
  out.margin_deg = bpx.margin_deg;
  // --------------------------------------------------------- subdivision
  Ctx C;
  C.P = &P;
  C.bp = bpx;
  int nthreads = bp.threads > 0 ? bp.threads : (int)std::max(1u, std::thread::hardware_concurrency());

  if (bpx.max_covering_cells > 0) {
    // the paper's coverings with cell budgets, merged (exact mode)
    std::vector<Sink> one(1);
    budget_super_covering(C, nthreads, one[0]);
    if (C.failed) {
      err = C.err;
      return C.err_code;
    }
    return finish_build(C, P, bpx, one, out, err, t0, n_polys);
  }
  std::vector<int32_t> all_polys;
  std::vector<Bref> all_bnd;
  std::vector<int32_t> all_edges;
  for (int p = 0; p < n_polys; p++) {
    all_bnd.push_back({p, (int32_t)all_edges.size(), P.e_off[p + 1] - P.e_off[p]});
    for (int e = P.e_off[p]; e < P.e_off[p + 1]; e++) all_edges.push_back(e);
  }
  std::vector<Work> frontier;
  Sink top;
  for (int face = 0; face < 6; face++) {
    Work w;
    w.face = face;
    w.level = 0;
    w.i = w.j = 0;
    w.box = inflate(cell_bounds(face, 0, 0, 0), bpx.margin_deg);
    std::vector<int32_t> none;
    classify(C, w.box, none, all_bnd, all_edges, w);
    frontier.push_back(std::move(w));
  }
  all_bnd.clear();
  all_edges.clear();
  // expand breadth-first until there is enough independent work
  std::vector<Work> tasks;
  while (!frontier.empty()) {
    std::vector<Work> next;
    for (Work &w : frontier) {
      if (!settle(C, w, top)) continue;
      for (int q = 0; q < 4; q++) {
        Work c;
        make_child(C, w, q, c);
        next.push_back(std::move(c));
      }
    }
    frontier.swap(next);
    if (frontier.size() >= (size_t)(64 * nthreads)) break;
  }
  tasks.swap(frontier);
  // one sink per task, gathered in task order: the index image does not
  // depend on the thread count or on scheduling
  std::vector<Sink> sinks(tasks.size());
  std::atomic<size_t> cursor{0};
  auto worker = [&](int) {
    for (;;) {
      size_t k = cursor.fetch_add(1);
      if (k >= tasks.size()) break;
      dfs(C, tasks[k], sinks[k]);
    }
  };
  std::vector<std::thread> pool;
  for (int t = 1; t < nthreads; t++) pool.emplace_back(worker, t);
  worker(0);
  for (auto &th : pool) th.join();
  tasks.clear();
  if (C.failed) {
    err = C.err;
    return C.err_code;
  }
  std::vector<Sink> all;
  all.reserve(sinks.size() + 1);
  all.push_back(std::move(top));
  for (Sink &k : sinks) all.push_back(std::move(k));
  return finish_build(C, P, bpx, all, out, err, t0, n_polys);
}

}  // namespace act
