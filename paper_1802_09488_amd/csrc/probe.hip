// probe.hip -- the GPU probe (Section III-E, Listings 2 and 3) for gfx950,
// and the C ABI around it.
//
// Per point (one lane each, grid-stride):
//   1. coalesced 16-byte load of (lat, lng) fp64;
//   2. domain check (non-finite / |lat| > 90 / |lng| > 180 -> no match);
//   3. fp64 projection lat/lng -> unit sphere -> cube face -> (u, v) ->
//      linear (s, t) -> 30-bit (i, j) (Section II, S2 paragraph);
//   4. the trie key is the leaf's quadtree path, 4 bits of i and 4 of j
//      per node (the Hilbert id of step 4 is computed only for
//      act_cell_ids, from a 4-levels-per-step state table held in LDS);
//   5. stage 1 (Listing 4): face -> root, per-face common prefix check;
//   6. stage 2 (Listing 5): comparison-free descent, 8 key bits per node,
//      until a payload, a LUT offset or the sentinel;
//   7. stage 3: decode the tagged entry (Section III-E, three cases);
//   8. true hits (and every reference in approximate mode) are output;
//      in exact mode a point whose cell has candidate references is
//      pending: its candidates are refined by the crossing-number test of
//      Section II with the ST_Covers boundary rule. By default the join
//      has two passes: each probe wave lists its pending points (index and
//      cell entry) in its own region of a workspace list, and a second
//      kernel refines them from the cells' local records. Refinement over
//      all edges (fp32 on origin-translated coordinates with a proven error
//      bound, fp64 + exact arithmetic for the edges the bound leaves
//      undecided) and batched joins mark pending points in a per-64-point
//      mask for the resolve kernel instead; or each wave queues its pending
//      points in LDS and refines them itself, 64 at a time;
//   9. out[i] = lowest matching id (or -1), further matches -> pair list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <unordered_map>
#include <string>
#include <vector>

#include "../../include/act.h"
#include "cellid.hpp"
#include "geom.hpp"
#include "index.hpp"

namespace act {

// ------------------------------------------------------------------ state

static thread_local std::string g_err;

static int fail(int code, const std::string &msg) {
  g_err = msg;
  return code;
}

#define HIP_TRY(expr)                                                              \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess)                                                          \
      return fail(ACT_E_HIP, std::string(#expr ": ") + hipGetErrorString(_e));     \
  } while (0)

struct DevImage {
  uint32_t *nodes = nullptr;  // trie entries, 32 bits each
  uint32_t *lut = nullptr;
  int32_t *eoff = nullptr;
  double2 *origin = nullptr;
  float *pm = nullptr;
  float4 *e32 = nullptr;
  double2 *e64 = nullptr;
  double2 *trig = nullptr;
  struct FaceDev *faces = nullptr;
  uint64_t *sink = nullptr;  // 64 bytes that the probe's idle lanes store to
  uint16_t *hinv = nullptr;  // inverse Hilbert table (joins of precomputed ids)
  double *normals = nullptr;  // ACT_GEOM_SPHERE: great-circle normal of each edge
  size_t bytes = 0;
};

// Per-stream scratch of exact-mode joins: the pending mask, one bit per
// point of a pass (a join longer than `cap` points runs in passes).
struct Workspace {
  uint64_t *mask = nullptr;
  int64_t cap = 0;  // points
  // the probe waves' pending lists (cell-local refinement): room for cap
  // points plus the ragged ends of up to kListWavesMax waves' regions
  uint2 *plist = nullptr;
  int64_t plist_cap = 0;
  uint32_t *pcount = nullptr;
  // batched joins: virtual point space of up to cap_groups 64-point groups
  uint64_t *bmask = nullptr, *gticks = nullptr;
  int32_t *group_batch = nullptr;
  int64_t *vstart = nullptr, *vhdr = nullptr;
  int64_t *vsorted = nullptr;  // batches' virtual starts in virtual order
  int32_t *vorder = nullptr;   // the batch at each position of that order
  int64_t cap_groups = 0;
  int32_t cap_batches = 0;
};

constexpr int64_t kDefaultPass = 1 << 24;
// Probe waves whose pending lists a workspace holds (grids up to 4096
// blocks; larger grids fall back to the pending mask).
constexpr int64_t kListWavesMax = 4096 * 16;
// Points per probe launch at most: tile indices are 32-bit (2^31 tiles of
// 64 points, plus the grid's waves, stay below 2^32).
constexpr int64_t kMaxLaunchPoints = 1ll << 37;

}  // namespace act

// Launch configuration used when a join leaves a knob at its default
// (set by act_tune; the built-in defaults otherwise).
struct act_launch {
  int32_t grid = 1024;
  int32_t lds_levels = -1;       // -1: deepest that fits
  int32_t points_per_lane = 2;
  int32_t refine = ACT_REFINE_LOCAL;
  int32_t pending = ACT_PENDING_KERNEL;
};

struct act_index {
  act::HostIndex host;
  act::DevImage dev;
  int device = -1;
  act_launch launch;  // written only by act_tune
  mutable std::mutex ws_mu;
  mutable std::unordered_map<void *, act::Workspace> ws;
};

namespace act {

// Per-face lookup data in LDS: root node, prefix level shift and the
// common prefix (i, j) >> (30 - Lp) shared by all of the face's cells.
struct FaceDev {
  int32_t root;  // node index, -1 if the face has no cells
  int32_t sh0;   // 30 - Lp
  uint32_t pi, pj;
};

// Kernel parameters (passed by value).
struct ProbeParams {
  const double2 *pts;
  int64_t n;
  int32_t *out;
  int64_t *pair_pt;
  int32_t *pair_poly;
  int64_t cap;
  int64_t *n_pairs;
  unsigned long long *counters;
  const uint32_t *nodes;  // trie entries (32-bit: all fit, see the builder)
  uint32_t node_bytes32;  // the entries' bytes when below 2^32 - 4096, else 0
  const uint32_t *lut;
  const int32_t *eoff;
  const double2 *origin;
  const float *pm;
  const float4 *e32;
  const double2 *e64;
  const double2 *trig;   // kTrigEntries (cos, sin) of whole degrees (device)
  const FaceDev *faces;  // 6 entries (device)
  const uint32_t *top32;  // nodes 1 .. n_d0 + n_d1 (the top levels, staged in LDS)
  int32_t n_lds_nodes;    // trie nodes 1 .. n_lds_nodes staged in LDS
  int32_t refine;
  const uint32_t *local;  // exact mode: base of the cell-local records (the LUT)
  uint64_t *mask;         // exact mode: pending points of this pass, bit per point
  uint2 *plist;           // or: each probe wave's pending points (index, code)
  uint32_t *pcount;       //   and how many each wave has
  uint32_t region;        //   entries per wave
  int64_t base;           // index of pts[0] in the caller's array (pair output)
  uint64_t *sink;         // target of the stores of lanes without a point
  // batched joins: the batches laid end to end in a virtual point space,
  // each starting at a multiple of 128 points
  const act_batch *batches;
  const int32_t *group_batch;  // batch of each 64-point group of that space
  const int64_t *vstart;       // first virtual point of each batch, [nb] = end
  const int64_t *vhdr;         // [0] virtual groups in use (0 on a bad call)
  uint64_t *gticks;            // optional: completion tick of each group
  // count joins: per-polygon number of covering points, accumulated in
  // `counts` (device, one per polygon), through a per-block LDS histogram of
  // hist_bins bins when the polygons fit it (0: straight to `counts`)
  unsigned long long *counts;
  int32_t hist_bins;
  // joins of precomputed cell ids: the level-30 ids of the points (the
  // points themselves, pts, are then read only to refine pending ones)
  const uint64_t *ids;
  const uint16_t *hinv;  // inverse Hilbert table, 1024 entries (device)
  // ACT_GEOM_SPHERE: edges are great-circle arcs with these normals (3
  // doubles per edge); candidates are refined over all of a polygon's arcs
  const double *normals;
};


constexpr int kBlock = 256;  // resolve kernels
// The probe runs 1024-thread blocks: one LDS copy of the top trie levels
// then serves 16 wavefronts, and two blocks fill a CU.
constexpr int kProbeBlock = 1024;
constexpr int kProbeWaves = kProbeBlock / 64;

// --------------------------------------------------------- device math
//
// The projection needs fp64 (level-30 cells are 2^-30 of a face wide) but
// only to ~1e-13 relative: the builder's conservative cell boxes carry a
// 1e-9 degree margin. The pieces below are written for the argument ranges
// that occur and cost far fewer instructions than general library routines.

// Angles are split at the nearest whole degree b: x = b + u, |u| <= 1/2
// degree. (cos b, sin b) come from a 361-entry table (b = -180 .. 180,
// computed on the host with the C library), and sin d, cos d (d = u pi/180)
// from short Taylor series in u, the degree-to-radian factor folded into
// the coefficients: cos d to the d^4 term (the first omitted term is below
// 7e-16), no quadrant logic. The join's sine stops at the d^3 term (the
// first omitted term is below 4.2e-13): it is the sine of an angle within
// 4.2e-13 radians (2.5e-11 degrees) of d, so the probe projects a point
// within 2.5e-11 degrees of the input in latitude and in longitude, which
// the 1e-9 degree margin of the cell classification covers 40 times, at any
// latitude. Cell ids (act_cell_ids) take the d^5 term too (first omitted
// term below 8e-19), so that they match the leaf cell of the point to
// within rounding. x - b is exact (Sterbenz's lemma, or b = 0).
constexpr int kTrigEntries = 361;
constexpr double kRad = 0.017453292519943295;  // pi / 180
constexpr double kSin3 = -kRad * kRad * kRad / 6.0;
constexpr double kSin5 = kRad * kRad * kRad * kRad * kRad / 120.0;
constexpr double kCos2 = -kRad * kRad / 2.0;
constexpr double kCos4 = kRad * kRad * kRad * kRad / 24.0;

template <bool LEAF_EXACT = false>
__device__ __forceinline__ void sincos_deg(const double2 *trig, double x, double &s, double &c) {
  const double b = rint(x);
  const double2 t = trig[(int)b + 180];  // (cos b, sin b)
  const double u = x - b;
  const double u2 = u * u;
  const double sd = u * (LEAF_EXACT ? fma(u2, fma(u2, kSin5, kSin3), kRad) : fma(u2, kSin3, kRad));
  const double cd = fma(u2, fma(u2, kCos4, kCos2), 1.0);
  s = fma(t.y, cd, t.x * sd);
  c = fma(t.x, cd, -(t.y * sd));
}

// 1 / a for a in [1/sqrt(3), 1]: hardware estimate + one Newton step. The
// estimate's relative error was measured below 2^-24 over 2^24 inputs of
// [0.5, 1], so the step leaves about 2^-48: the cell coordinates then err by
// far less than the 1e-9 degree margin of the cell classification.
__device__ __forceinline__ double rcp_nr(double a) {
  const double r = __builtin_amdgcn_rcp(a);
  return fma(r, fma(-a, r, 1.0), r);
}

// Linear st transform of a face coordinate w = c / major, w in [-1, 1], as
// a 30-bit cell coordinate floor(2^30 (1 + w) / 2), clamped; `r29` is
// 2^29 / major.
__device__ __forceinline__ uint32_t leaf_coord(double c, double r29) {
  const int32_t i = (int32_t)fma(c, r29, 536870912.0);
  return min((uint32_t)max(i, 0), (1u << 30) - 1u);
}

// Steps 2-3: leaf cell coordinates (face, i, j) of a point; false for
// points that are not finite or outside |lat| <= 90, |lng| <= 180.
// The face is the axis of the largest |coordinate| (ties go to the lower
// axis: x before y before z) and its sign; (u, v) are the two other
// coordinates in cyclic axis order divided by that magnitude.
template <bool LEAF_EXACT = false>
__device__ __forceinline__ bool project(const double2 *trig, double lat, double lng,
                                        uint32_t &face, uint32_t &i, uint32_t &j) {
  if (!(fabs(lat) <= 90.0 && fabs(lng) <= 180.0)) return false;
  double sp, cp, sl, cl;
  sincos_deg<LEAF_EXACT>(trig, lat, sp, cp);
  sincos_deg<LEAF_EXACT>(trig, lng, sl, cl);
  const double x = cp * cl, y = cp * sl, z = sp;
  const bool xmaj = fabs(x) >= fabs(y);
  const double mxy = fmax(fabs(x), fabs(y));
  const bool polar = fabs(z) > mxy;
  // (a select, not fmax: fmax would first quiet NaNs, which cannot occur)
  const double r29 = rcp_nr(polar ? fabs(z) : mxy) * 536870912.0;
  // the major coordinate is at least 1/sqrt(3) in magnitude, so its sign
  // bit (bit 31 of the high word) says whether it is negative
  const uint32_t hs = polar ? (uint32_t)__double2hiint(z)
                            : (uint32_t)__double2hiint(xmaj ? x : y);
  // the face is usually the same for the whole wavefront (regional data):
  // then a wave-uniform branch picks the coordinates without selects
  const uint32_t f = (polar ? 2u : (xmaj ? 0u : 1u)) + (hs >> 31) * 3u;
  const uint32_t f0 = __builtin_amdgcn_readfirstlane(f);
  if (__ballot(f != f0) == 0) {
    face = f0;
    if (f0 == 0u || f0 == 3u) {
      i = leaf_coord(y, r29);
      j = leaf_coord(z, r29);
    } else if (f0 == 1u || f0 == 4u) {
      i = leaf_coord(z, r29);
      j = leaf_coord(x, r29);
    } else {
      i = leaf_coord(x, r29);
      j = leaf_coord(y, r29);
    }
    return true;
  }
  // minor coordinates in axis order: x face (y, z), y face (z, x), z face (x, y)
  const double c1 = polar ? x : (xmaj ? y : z);
  const double c2 = polar ? y : (xmaj ? z : x);
  face = f;
  i = leaf_coord(c1, r29);
  j = leaf_coord(c2, r29);
  return true;
}

// One Hilbert table step: 4 levels starting below bit `sh` of (i, j).
// `st` holds the curve state << 8; returns the 4 digits (one key byte).
__device__ __forceinline__ uint32_t hstep(const uint16_t *htab, uint32_t &st, uint32_t i,
                                          uint32_t j, int sh) {
  const uint32_t ent = htab[st | (((i >> sh) & 15u) << 4) | ((j >> sh) & 15u)];
  st = ent & 0x300u;
  return ent & 255u;
}

// Full 60-bit Hilbert position of a leaf (32 padded levels, 8 steps).
__device__ __forceinline__ uint64_t hilbert60(const uint16_t *htab, uint32_t i, uint32_t j) {
  uint32_t st = 0, hi = 0, lo = 0;
#pragma unroll
  for (int sh = 28; sh >= 16; sh -= 4) hi = (hi << 8) | hstep(htab, st, i, j, sh);
#pragma unroll
  for (int sh = 12; sh >= 0; sh -= 4) lo = (lo << 8) | hstep(htab, st, i, j, sh);
  return ((uint64_t)hi << 32) | lo;
}

// --------------------------------------------------------- wave helpers

__device__ __forceinline__ uint64_t ballot(bool b) { return __ballot(b); }

__device__ __forceinline__ int lane_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// Orders LDS traffic of one wavefront (its lanes run in lockstep).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One edge of the crossing-number test. fp32 tier on origin-translated
// coordinates; edges it cannot decide go to the exact fp64 test.
// Returns 0 (no effect), 1 (toggle parity), 2 (point on the edge).
// fp32 edges are stored oriented upward (g.y <= g.w): the point is level
// with the edge's half-open y-range [ya, yb) exactly when ya <= py < yb, and
// the ray crosses it when the point lies left of the edge (orient > 0).
// Strict comparisons of rounded values imply the same strict order of the
// exact values; equal rounded values go to the exact test.
template <int FULL>
__device__ __forceinline__ int edge_fp32_then_exact(const ProbeParams &P, int e, float4 g,
                                                    float qx, float qy, float eta, double px,
                                                    double py, uint32_t &c_fp64,
                                                    uint32_t &c_exact) {
  if (g.y > qy || g.w < qy) return 0;  // strictly below / above the edge
  if (g.y < qy && g.w > qy) {           // strictly inside the y-range
    const int s = orient_sign_fp32_filter(g.x, g.y, g.z, g.w, qx, qy, eta);
    if (s != 0) return s > 0 ? 1 : 0;
  }
  const double2 A = P.e64[2 * e], B = P.e64[2 * e + 1];
  if (FULL == 2) {
    c_fp64++;
    if (orient_sign_fp64_filter(A.x, A.y, B.x, B.y, px, py) == 0) c_exact++;
  }
  return edge_test_exact(A.x, A.y, B.x, B.y, px, py);
}

template <int FULL>
__device__ __forceinline__ int edge_fp64(const ProbeParams &P, int e, double px, double py,
                                         uint32_t &c_fp64, uint32_t &c_exact) {
  const double2 A = P.e64[2 * e], B = P.e64[2 * e + 1];
  if ((A.y > py && B.y > py) || (A.y < py && B.y < py)) return 0;
  if (FULL == 2) {
    c_fp64++;
    if (orient_sign_fp64_filter(A.x, A.y, B.x, B.y, px, py) == 0) c_exact++;
  }
  return edge_test_exact(A.x, A.y, B.x, B.y, px, py);
}

// Unit vector of (lat, lng) degrees, with the full sine series: the
// refinement's sign tests need the point itself, not one within the cell
// margin.
__device__ __forceinline__ void unit_vector(const double2 *trig, double lat, double lng,
                                            double (&q)[3]) {
  double sp, cp, sl, cl;
  sincos_deg<true>(trig, lat, sp, cp);
  sincos_deg<true>(trig, lng, sl, cl);
  q[0] = cp * cl;
  q[1] = cp * sl;
  q[2] = sp;
}

// One edge of the spherical crossing test (ACT_GEOM_SPHERE): the arc from the
// point north along its meridian to the pole. Returns 0 (no effect), 1
// (toggle) or 2 (the point is a vertex or on the arc). The meridian meets
// the edge when the point's longitude lies in the edge's half-open range;
// it crosses it when the point and the pole are on opposite sides of the
// edge's great circle: det = q . (a x b) has the sign opposite to that of
// the pole's, which is the sign of lng_b - lng_a. Edges along a meridian are
// only touched.
__device__ __forceinline__ int edge_sphere(const ProbeParams &P, int e, double plat, double plng,
                                           const double (&q)[3]) {
  const double2 A = P.e64[2 * e], B = P.e64[2 * e + 1];  // (lng, lat)
  if ((plat == A.y && plng == A.x) || (plat == B.y && plng == B.x)) return 2;
  if (A.x == B.x)
    return plng == A.x && plat >= fmin(A.y, B.y) && plat <= fmax(A.y, B.y) ? 2 : 0;
  const double lo = fmin(A.x, B.x), hi = fmax(A.x, B.x);
  if (plng < lo || plng > hi) return 0;
  const double *n = P.normals + 3 * (size_t)e;
  const double det = q[0] * n[0] + q[1] * n[1] + q[2] * n[2];
  if (det == 0.0) return 2;
  if (plng == hi) return 0;
  return (det > 0.0) != (B.x > A.x) ? 1 : 0;
}

// Whole-wave point-in-polygon test of one (point, polygon) pair: lane l
// takes edges e0 + l, e0 + l + 64, ...; crossing parity = parity of the
// popcounts of the toggle ballots; any lane on an edge decides "covered".
// The next chunk of edges is loaded while the current one is tested. Must be
// called by all 64 lanes with wave-uniform arguments.
template <int FULL>
__device__ bool wave_covers(const ProbeParams &P, int poly, double lat, double lng, int lane,
                            uint32_t &c_fp64, uint32_t &c_exact) {
  const int e0 = P.eoff[poly], e1 = P.eoff[poly + 1];
  const double px = lng, py = lat;
  uint32_t par = 0;
  bool on = false;
  if (P.normals) {  // spherical edges
    double q[3];
    unit_vector(P.trig, lat, lng, q);
    for (int base = e0; base < e1; base += 64) {
      const int e = base + lane;
      const int r = e < e1 ? edge_sphere(P, e, lat, lng, q) : 0;
      on |= ballot(r == 2) != 0;
      par ^= (uint32_t)__popcll(ballot(r == 1));
    }
  } else if (P.refine != ACT_REFINE_FP64) {
    const double2 o = P.origin[poly];
    const float qx = (float)(px - o.x), qy = (float)(py - o.y);
    const float eta = tier1_eta(fmaxf(P.pm[poly], fmaxf(fabsf(qx), fabsf(qy))));
    float4 nxt = e0 + lane < e1 ? P.e32[e0 + lane] : make_float4(0.f, 0.f, 0.f, 0.f);
    for (int base = e0; base < e1; base += 64) {
      const int e = base + lane;
      const float4 g = nxt;
      if (e + 64 < e1) nxt = P.e32[e + 64];
      const int r = e < e1 ? edge_fp32_then_exact<FULL>(P, e, g, qx, qy, eta, px, py, c_fp64,
                                                         c_exact)
                           : 0;
      on |= ballot(r == 2) != 0;
      par ^= (uint32_t)__popcll(ballot(r == 1));
    }
  } else {
    for (int base = e0; base < e1; base += 64) {
      const int e = base + lane;
      const int r = e < e1 ? edge_fp64<FULL>(P, e, px, py, c_fp64, c_exact) : 0;
      on |= ballot(r == 2) != 0;
      par ^= (uint32_t)__popcll(ballot(r == 1));
    }
  }
  return on || (par & 1u) != 0;
}

// Lowest match goes to out[i]; every other match becomes a pair (PAIRS:
// only kernels built with pair output emit them, so the lean kernels of
// plain joins carry none of its registers).
template <bool PAIRS>
struct Hits {
  int32_t best = -1;
  __device__ __forceinline__ void add(const ProbeParams &P, int64_t i, int32_t poly) {
    if (best < 0) {
      best = poly;
      return;
    }
    const int32_t other = poly < best ? best : poly;
    best = poly < best ? poly : best;
    if (PAIRS && P.pair_pt) {
      const unsigned long long k = atomicAdd((unsigned long long *)P.n_pairs, 1ull);
      if ((int64_t)k < P.cap) {
        P.pair_pt[k] = i;
        P.pair_poly[k] = other;
      }
    }
  }
};

// One (point, polygon) match of a count join: a histogram bin in LDS, or
// the polygon's global counter.
__device__ __forceinline__ void count_add(const ProbeParams &P, uint32_t *s_hist, uint32_t poly) {
  if (s_hist)
    atomicAdd(s_hist + poly, 1u);
  else
    atomicAdd(P.counts + poly, 1ull);
}

// Steps 5-6: prefix check (Listing 4) and comparison-free descent
// (Listing 5). Each node consumes 4 levels of the cell's quadtree path, its
// key byte being (4 bits of i, 4 bits of j). The first LDS_DEPTH node levels
// are read from the LDS copy of nodes 1 .. n_lds_nodes (breadth-first
// numbering puts the top levels first).
template <int LDS_DEPTH>
__device__ __forceinline__ uint64_t lookup(const ProbeParams &P, const uint32_t *s_nodes,
                                           const FaceDev &F, uint32_t i, uint32_t j,
                                           uint32_t &reads) {
  const int root = F.root;
  int sh = F.sh0;
  if (root < 0 || (i >> sh) != F.pi || (j >> sh) != F.pj) return 0;
  uint64_t node = (uint64_t)root, e;
#pragma unroll
  for (int d = 0; d < LDS_DEPTH; d++) {
    sh -= 4;
    e = s_nodes[(node - 1) * 256 + node_slot(i, j, sh)];  // high 32 bits are zero
    reads++;
    if ((e & kTagMask) != kTagPtr || e == 0) return e;
    node = e >> 2;
  }
  for (;;) {
    sh -= 4;
    e = P.nodes[node * 256 + node_slot(i, j, sh)];
    reads++;
    if ((e & kTagMask) != kTagPtr || e == 0) return e;
    node = e >> 2;
  }
}

// out[] of a pending point until the resolve kernel overwrites it: -3 - the
// offset of the cell's lookup-table list (offsets stay below 2^30, the
// builder's bound on the table), or kPending when the cell's references are
// inline (the resolver then repeats the descent).
constexpr int32_t kPending = -2;

__device__ __forceinline__ bool is_child(uint64_t e) { return (e & kTagMask) == kTagPtr && e != 0; }

// Streaming accesses: each point is read once and each output written once,
// so they bypass the caches' retention (nontemporal), leaving L2 to the
// trie nodes that every point's descent revisits. A tile's points and
// outputs are accessed through a buffer resource spanning exactly the
// tile's points (base and size are wave-uniform): the hardware's range
// check turns the accesses of lanes past the tile's end into reads of zero
// and dropped stores, so every lane issues them without any address
// clamping or masking, and the compiler's waits for the loads in flight
// stay exact. (Raw buffer, stride 0; the third descriptor word is the
// 32-bit data format the gfx9 family expects; aux 2 = nontemporal.)
constexpr int kBufferFlags = 0x00020000;
constexpr int kBufferNT = 2;
constexpr int kBufferOutOfRange = 0x40000000;  // beyond every tile and list buffer
// beyond the trie's entries: the buffer path is taken for tries below this
constexpr uint32_t kNodeBuffer32Max = 0xfffff000u;
constexpr int kNodeOutOfRange = (int)0xfffff000u;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t tile_buffer(const void *base, int32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes, kBufferFlags);
}

typedef int act_int4_v __attribute__((ext_vector_type(4)));
typedef int act_int2_v __attribute__((ext_vector_type(2)));

// Steps 5-6 for NP points of a lane at once, split into the parts of the
// probe's pipeline: the prefix check and the LDS-staged levels
// (descend_lds), one global node level (issue_level / take_level) and the
// remaining global levels (descend_rest). The descents run side by side,
// so each step issues up to NP independent loads.
//
// Node level d below a face's prefix (d = 0 .. 7; the builder keeps every
// trie within 8 levels of its prefix) is keyed by the d-th nibbles of i and
// j under the prefix. Those key bytes are gathered once per point into two
// words: with a, b = i, j shifted so that their first nibble under the
// prefix is the top one, `ev` holds the bytes of the even levels (level
// 2k in byte 3 - k) and `od` those of the odd ones, so a level's key is one
// bit-field extract at an offset known at compile time. All lanes of a wave
// walk the levels in step, so the level index is uniform.
//
// Written without branches: a lane whose descent has ended keeps its entry
// and its last node, whose LDS copy it keeps reading harmlessly (a lane that
// never started reads node 1, the first LDS-staged node), and at the global
// levels it reads nothing (issue_level), so the wave never splits. Device
// entries are 32-bit;
// a node is carried as its pointer entry (index << 2), so its byte offset
// is the entry << 8.
template <int NP>
struct Descent {
  uint32_t ev[NP], od[NP];
  uint32_t node[NP];
  uint32_t e[NP];
  bool act[NP];
};

template <int D>
__device__ __forceinline__ uint32_t level_key(uint32_t ev, uint32_t od) {
  return ((D & 1 ? od : ev) >> (24 - 8 * (D >> 1))) & 255u;
}

// One level's entry v of a lane: record it while the descent is live, and
// follow it if it is a child pointer (tag 00, nonzero).
template <int NP>
__device__ __forceinline__ void step_level(Descent<NP> &D, int p, uint32_t v, uint32_t &reads) {
  reads += D.act[p];
  D.e[p] = D.act[p] ? v : D.e[p];
  const bool ptr = D.act[p] & ((v & 3u) == 0u) & (v != 0u);
  D.node[p] = ptr ? v : D.node[p];
  D.act[p] = ptr;
}

template <int LDS_DEPTH, int NP>
__device__ __forceinline__ void descend_lds(const uint32_t *s_nodes, const FaceDev *s_face,
                                            const uint32_t (&face)[NP], const uint32_t (&ci)[NP],
                                            const uint32_t (&cj)[NP], const bool (&valid)[NP],
                                            Descent<NP> &D, uint32_t &reads) {
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const FaceDev F = s_face[face[p]];
    D.act[p] = valid[p] & (F.root >= 0) & ((ci[p] >> F.sh0) == F.pi) &
               ((cj[p] >> F.sh0) == F.pj);
    // i, j << (32 - sh0): the bits under the prefix at the top (0 when the
    // prefix is the leaf level: such a root's entries are all one cell)
    const uint32_t a = __builtin_amdgcn_alignbit(ci[p], 0u, (uint32_t)F.sh0);
    const uint32_t b = __builtin_amdgcn_alignbit(cj[p], 0u, (uint32_t)F.sh0);
    D.ev[p] = (a & 0xf0f0f0f0u) | ((b >> 4) & 0x0f0f0f0fu);
    D.od[p] = ((a << 4) & 0xf0f0f0f0u) | (b & 0x0f0f0f0fu);
    D.node[p] = D.act[p] ? (uint32_t)F.root << 2 : (LDS_DEPTH > 0 ? 1u << 2 : 0u);
    D.e[p] = 0u;
  }
  // s_nodes holds nodes 1 .. n_lds_nodes, which include every node of the
  // LDS-staged levels
  const uint32_t *s_base = s_nodes - 256;
#pragma unroll
  for (int d = 0; d < LDS_DEPTH; d++) {
#pragma unroll
    for (int p = 0; p < NP; p++) {
      const uint32_t key = d == 0 ? level_key<0>(D.ev[p], D.od[p]) : level_key<1>(D.ev[p], D.od[p]);
      step_level<NP>(D, p, s_base[(D.node[p] << 6) | key], reads);
    }
  }
}

// Global node level D_: a buffer over the trie's entries (32-bit offsets)
// when they span under 4 GiB, else 64-bit addresses. (The flag is uniform,
// and both paths issue the same loads, so the waits stay exact.) Lanes
// whose descent has ended must not each fetch a line of their last node:
// their buffer offset is out of range (no memory access, zero returned),
// or their address is node 0's first entry (one line for all of them).
template <int NP, int D_>
__device__ __forceinline__ void issue_level(const ProbeParams &P, const Descent<NP> &D,
                                            uint32_t (&x)[NP]) {
  if (P.node_bytes32) {
    const __amdgpu_buffer_rsrc_t nb = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<uint32_t *>(P.nodes), (short)0, (int)P.node_bytes32, kBufferFlags);
#pragma unroll
    for (int p = 0; p < NP; p++) {
      const uint32_t off = (D.node[p] << 8) | (level_key<D_>(D.ev[p], D.od[p]) << 2);
      x[p] = __builtin_amdgcn_raw_buffer_load_b32(nb, D.act[p] ? (int)off : kNodeOutOfRange, 0, 0);
    }
  } else {
#pragma unroll
    for (int p = 0; p < NP; p++) {
      const uint64_t k = ((uint64_t)D.node[p] << 6) | level_key<D_>(D.ev[p], D.od[p]);
      x[p] = P.nodes[D.act[p] ? k : 0u];
    }
  }
}

template <int NP>
__device__ __forceinline__ void take_level(Descent<NP> &D, const uint32_t (&x)[NP],
                                           uint32_t &reads) {
#pragma unroll
  for (int p = 0; p < NP; p++) step_level<NP>(D, p, x[p], reads);
}

// Levels D_ .. 7, while any of the lane's descents is live.
template <int NP, int D_>
__device__ __forceinline__ void descend_rest(const ProbeParams &P, Descent<NP> &D,
                                             uint32_t &reads) {
  if constexpr (D_ < 8) {
    bool any = false;
#pragma unroll
    for (int p = 0; p < NP; p++) any |= D.act[p];
    if (!any) return;
    uint32_t x[NP];
    issue_level<NP, D_>(P, D, x);
    take_level<NP>(D, x, reads);
    descend_rest<NP, D_ + 1>(P, D, reads);
  }
}

// Where a tile's points live: its first point, its output, how many of
// the tile's 64 NP points exist (0 .. 64 NP), and the caller's index of its
// first point (pair output; single joins only). A single join's tiles
// are consecutive; a batched join's tile lies inside one batch (batches
// start at multiples of 128 virtual points).
struct TileRef {
  const double2 *pts;
  int32_t *out;
  int32_t n;
  int64_t gi;
  const uint64_t *ids;  // joins of precomputed ids: the tile's first id
};

// Tile indices are 32-bit (a launch covers fewer than 2^32 tiles), so the
// wave-uniform loop bookkeeping stays in scalar registers.
template <bool BATCHED, int NP>
__device__ __forceinline__ TileRef tile_ref(const ProbeParams &P, uint32_t tile) {
  constexpr int TILE = 64 * NP;
  TileRef r;
  int64_t rest;
  if (!BATCHED) {
    const int64_t s = (int64_t)tile * TILE;
    r.pts = P.pts + s;
    r.out = P.out + s;
    rest = P.n - s;
    r.gi = P.base + s;
    r.ids = P.ids + s;
  } else {
    const int32_t b = P.group_batch[(int64_t)tile * NP];
    const int64_t off = (int64_t)tile * TILE - P.vstart[b];
    const act_batch d = P.batches[b];
    r.pts = (const double2 *)d.d_points + off;
    r.out = d.d_out + off;
    rest = d.n - off;
    r.gi = -1;
    r.ids = nullptr;
  }
  r.n = (int32_t)std::max<int64_t>(0, std::min<int64_t>(rest, TILE));
  return r;
}

// References of a pending point's cell: true ids first, then candidates
// (each with its cell-local record offset when the list carries one).
struct RefList {
  uint32_t off = 0, nt = 0, nc = 0;
  uint32_t a = 0, b = 0;  // inline references (true ones first)
  bool lut = false;
  __device__ __forceinline__ uint32_t true_id(const ProbeParams &P, uint32_t r) const {
    return lut ? P.lut[off + 1 + r] : (r == 0 ? a : b);
  }
  __device__ __forceinline__ uint32_t cand_id(const ProbeParams &P, uint32_t r) const {
    return lut ? P.lut[off + 2 + nt + r] : (nt + r == 0 ? a : b);
  }
  __device__ __forceinline__ uint32_t cand_loc(const ProbeParams &P, uint32_t r) const {
    return lut && P.local ? P.lut[off + 2 + nt + nc + r] : 0xffffffffu;
  }
};

// The list's first words are read together (the device copy of the table
// is padded, so this stays in bounds): lists with up to two true hits need
// no second, dependent read for their candidate count.
__device__ __forceinline__ RefList lut_refs(const ProbeParams &P, uint32_t off) {
  RefList L;
  L.lut = true;
  L.off = off;
  const uint32_t w0 = P.lut[off], w1 = P.lut[off + 1], w2 = P.lut[off + 2], w3 = P.lut[off + 3];
  L.nt = w0;
  L.nc = w0 == 0 ? w1 : (w0 == 1 ? w2 : (w0 == 2 ? w3 : P.lut[off + 1 + w0]));
  return L;
}

// The references of a cell entry (a lookup-table list, or one or two inline
// references, interior ones first).
__device__ __forceinline__ RefList entry_refs(const ProbeParams &P, uint64_t e) {
  const uint32_t tag = (uint32_t)(e & kTagMask);
  if (e == 0 || tag == kTagPtr) return RefList();
  if (tag == kTagLut) return lut_refs(P, (uint32_t)(e >> 2));
  RefList L;
  const uint32_t v0 = (uint32_t)((e >> 2) & 0x7fffffffu), v1 = (uint32_t)((e >> 33) & 0x7fffffffu);
  const int n = tag == kTagTwo ? 2 : 1;
  uint32_t slot[2];
  int k = 0;
  for (int t = 1; t >= 0; t--) {  // interior references first
    if ((v0 & 1u) == (uint32_t)t) slot[k++] = v0 >> 1;
    if (n > 1 && (v1 & 1u) == (uint32_t)t) slot[k++] = v1 >> 1;
  }
  L.a = slot[0];
  L.b = n > 1 ? slot[1] : 0u;
  L.nt = (v0 & 1u) + (n > 1 ? (v1 & 1u) : 0u);
  L.nc = (uint32_t)n - L.nt;
  return L;
}

// The pending point's references in a two-pass join: from the list offset
// the probe left in out[], or by repeating the lookup (inline entries).
__device__ __forceinline__ RefList pending_refs(const ProbeParams &P, int32_t code, double lat,
                                                double lng, uint32_t &reads) {
  if (code <= -3) return lut_refs(P, (uint32_t)(-3 - code));
  uint32_t face, ci, cj;
  uint64_t e = 0;
  if (project(P.trig, lat, lng, face, ci, cj))
    e = lookup<0>(P, nullptr, P.faces[face], ci, cj, reads);
  return entry_refs(P, e);
}

// All edges of a polygon tested by one lane in fp64 (+ exact): used only
// for a candidate without a cell-local record.
template <int FULL>
__device__ bool lane_covers(const ProbeParams &P, int poly, double lat, double lng,
                            uint32_t &c_fp64, uint32_t &c_exact) {
  uint32_t par = 0;
  if (P.normals) {  // spherical edges
    double q[3];
    unit_vector(P.trig, lat, lng, q);
    for (int e = P.eoff[poly]; e < P.eoff[poly + 1]; e++) {
      const int r = edge_sphere(P, e, lat, lng, q);
      if (r == 2) return true;
      par ^= (uint32_t)r;
    }
    return par != 0;
  }
  for (int e = P.eoff[poly]; e < P.eoff[poly + 1]; e++) {
    const int r = edge_fp64<FULL>(P, e, lng, lat, c_fp64, c_exact);
    if (r == 2) return true;
    par ^= (uint32_t)r;
  }
  return par != 0;
}

template <int FULL>
__device__ __forceinline__ void flush_counters(const ProbeParams &P, const uint32_t *c) {
  if (FULL != 2 || !P.counters) return;
  static constexpr int ids[7] = {ACT_CNT_SOLELY_TRUE, ACT_CNT_CAND_POINTS, ACT_CNT_CANDIDATES,
                                 ACT_CNT_EDGES, ACT_CNT_EDGE_FP64, ACT_CNT_EDGE_EXACT,
                                 ACT_CNT_LUT_READS};
  for (int k = 0; k < 7; k++)
    if (c[k]) atomicAdd(P.counters + ids[k], (unsigned long long)c[k]);
}

// Pending points of a resolve block range: kRangeWords mask words (64
// points each, of the pass or of a batched join's virtual space), one per
// thread. The block compacts their set bits into an LDS list (block-wide
// prefix sum of the popcounts) and hands the list out one point per
// thread; bits beyond the list's capacity (more than a quarter of the
// range's points pending) stay with the thread that read them.
constexpr int kRangeWords = 256;
constexpr int kResolveBlock = 256;
constexpr int kListCap = 4096;

struct PendingIter {
  int k, total;
  uint64_t m;    // bits of this thread's word not in the list
  int64_t w;     // this thread's mask word
  int64_t base;  // first point of the block's range
  __device__ __forceinline__ bool next(const uint16_t *s_list, int64_t &v) {
    if (k < total) {
      v = base + s_list[k];
      k += kResolveBlock;
      return true;
    }
    if (m) {
      v = w * 64 + (__ffsll((long long)m) - 1);
      m &= m - 1;
      return true;
    }
    return false;
  }
};

__device__ __forceinline__ PendingIter gather_pending(const ProbeParams &P, int64_t blk,
                                                      int64_t nwords, uint16_t *s_list,
                                                      uint32_t *s_wave) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  PendingIter it;
  it.base = blk * kRangeWords * 64;
  it.w = blk * kRangeWords + threadIdx.x;
  uint64_t m = it.w < nwords ? P.mask[it.w] : 0ull;
  const uint32_t c = (uint32_t)__popcll(m);
  uint32_t incl = c;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t v = __shfl_up(incl, d);
    if (lane >= d) incl += v;
  }
  if (lane == 63) s_wave[wid] = incl;
  __syncthreads();
  uint32_t pos = incl - c, total = 0;
  for (int k = 0; k < kRangeWords / 64; k++) {
    if (k < wid) pos += s_wave[k];
    total += s_wave[k];
  }
  while (m && pos < (uint32_t)kListCap) {
    s_list[pos++] = (uint16_t)((threadIdx.x << 6) | (__ffsll((long long)m) - 1));
    m &= m - 1;
  }
  __syncthreads();
  it.m = m;
  it.k = threadIdx.x;
  it.total = (int)min(total, (uint32_t)kListCap);
  return it;
}

// A pending point: where it is, where its result goes, and the caller's
// index of it (pair output; single joins only).
struct PointRef {
  const double2 *pt;
  int32_t *out;
  int64_t gi;
};

template <bool BATCHED>
__device__ __forceinline__ PointRef point_ref(const ProbeParams &P, int64_t v) {
  PointRef r;
  if (!BATCHED) {
    r.pt = P.pts + v;
    r.out = P.out + v;
    r.gi = P.base + v;
  } else {
    const int32_t b = P.group_batch[v >> 6];
    const int64_t k = v - P.vstart[b];
    const act_batch d = P.batches[b];
    r.pt = (const double2 *)d.d_points + k;
    r.out = d.d_out + k;
    r.gi = -1;
  }
  return r;
}

// A batched join's group is complete once its last pending point is (the
// probe stores each group's tick when its tile finishes; a pending point
// resolved later raises it).
template <bool BATCHED>
__device__ __forceinline__ void point_done(const ProbeParams &P, int64_t v) {
  if (BATCHED && P.gticks)
    atomicMax((unsigned long long *)P.gticks + (v >> 6), (unsigned long long)wall_clock64());
}

// Step 8 with cell-local refinement for one pending point v (an index of
// the pass, or of a batched join's virtual space) whose cell code is
// `code`: true references are hits, and each candidate is decided from its
// cell-local record (all of the polygon's edges for a candidate without
// one). Counters go to c: solely-true, candidate points, candidates, edges,
// fp64 edges, exact edges, lookup-table reads.
// `entry`: the cell's entry when the caller has it (fused probe), else the
// code the probe left in out[] (two-pass join).
// COUNT: a count join's resolve, which adds each match to the polygon's
// counter instead of writing out[].
template <int FULL, bool BATCHED, bool ENTRY, bool COUNT = false>
__device__ __forceinline__ void resolve_point(const ProbeParams &P, int64_t v, uint64_t entry,
                                              uint32_t (&c)[7], uint32_t &c_reads,
                                              uint32_t *s_hist = nullptr) {
  const PointRef R = point_ref<BATCHED>(P, v);
  const double2 pt = *R.pt;
  const RefList L = ENTRY ? entry_refs(P, entry)
                          : pending_refs(P, (int32_t)(uint32_t)entry, pt.x, pt.y, c_reads);
  Hits<(FULL >= 1)> hits;
  for (uint32_t r = 0; r < L.nt; r++) {
    if (COUNT)
      count_add(P, s_hist, L.true_id(P, r));
    else
      hits.add(P, R.gi, (int32_t)L.true_id(P, r));
  }
  for (uint32_t r = 0; r < L.nc; r++) {
    const int32_t poly = (int32_t)L.cand_id(P, r);
    const uint32_t loc = L.cand_loc(P, r);
    bool cov;
    if (loc != 0xffffffffu) {
      cov = local_record_covers(P.local + loc, pt.y, pt.x);
      if (FULL == 2) c[3] += P.local[loc] + (P.local[loc + 1] & 0x7fffffffu);
    } else {
      cov = lane_covers<FULL>(P, poly, pt.x, pt.y, c[4], c[5]);
      if (FULL == 2) c[3] += (uint32_t)(P.eoff[poly + 1] - P.eoff[poly]);
    }
    if (cov) {
      if (COUNT)
        count_add(P, s_hist, (uint32_t)poly);
      else
        hits.add(P, R.gi, poly);
    }
  }
  if (!COUNT) *R.out = hits.best;
  point_done<BATCHED>(P, v);
  if (FULL == 2) {
    c[0] += L.nc == 0 && L.nt > 0;
    c[1] += L.nc > 0;
    c[2] += L.nc;
    c[6] += L.lut;
  }
}

// The second pass of a two-pass exact join: resolve the pending points of
// the mask, block range by block range. LOCAL: each thread decides its
// point's candidates from their cell-local records. Otherwise (refinement
// over all of a polygon's edges) lanes gather their points' candidates and
// the whole wave tests one (point, polygon) pair at a time (lanes over
// edges, see wave_covers); in every round each lane with work offers its
// next candidate.
template <bool LOCAL, int FULL, bool BATCHED>
__global__ __launch_bounds__(kResolveBlock) void resolve_kernel(ProbeParams P,
                                                                 int64_t nwords_arg) {
  __shared__ uint16_t s_list[kListCap];
  __shared__ uint32_t s_wave[kRangeWords / 64];
  const int64_t nwords = BATCHED ? P.vhdr[0] : nwords_arg;
  uint32_t c[7] = {0, 0, 0, 0, 0, 0, 0}, c_reads = 0;
  for (int64_t blk = blockIdx.x; blk * kRangeWords < nwords; blk += gridDim.x) {
    PendingIter it = gather_pending(P, blk, nwords, s_list, s_wave);
    int64_t v = 0;
    if (LOCAL) {
      while (it.next(s_list, v))
        resolve_point<FULL, BATCHED, false>(P, v, (uint32_t)*point_ref<BATCHED>(P, v).out, c,
                                             c_reads);
    } else {
      const int lane = threadIdx.x & 63;
      bool have = false, more = true;
      double lat = 0.0, lng = 0.0;
      RefList L;
      PointRef R{nullptr, nullptr, 0};
      uint32_t r = 0;
      Hits<(FULL >= 1)> hits;
      for (;;) {
        if (!have && more) {
          more = it.next(s_list, v);
          if (more) {
            R = point_ref<BATCHED>(P, v);
            const double2 pt = *R.pt;
            lat = pt.x;
            lng = pt.y;
            L = pending_refs(P, *R.out, lat, lng, c_reads);
            hits = Hits<(FULL >= 1)>();
            for (uint32_t t = 0; t < L.nt; t++) hits.add(P, R.gi, (int32_t)L.true_id(P, t));
            r = 0;
            have = true;
            if (FULL == 2) {
              c[0] += L.nc == 0 && L.nt > 0;
              c[1] += L.nc > 0;
              c[2] += L.nc;
              c[6] += L.lut;
            }
          }
        }
        if (have && r >= L.nc) {
          *R.out = hits.best;
          have = false;
        }
        uint64_t todo = ballot(have);
        if (!todo) {
          if (!ballot(more)) break;
          continue;
        }
        const int32_t poly = have ? (int32_t)L.cand_id(P, r) : 0;
        while (todo) {
          const int src = __ffsll((long long)todo) - 1;
          todo &= todo - 1;
          const int32_t q = __shfl(poly, src);
          const double qlat = __shfl(lat, src), qlng = __shfl(lng, src);
          if (FULL == 2 && lane == 0) c[3] += (uint32_t)(P.eoff[q + 1] - P.eoff[q]);
          const bool cov = wave_covers<FULL>(P, q, qlat, qlng, lane, c[4], c[5]);
          if (lane == src && cov) hits.add(P, R.gi, q);
        }
        if (have) r++;
      }
    }
    __syncthreads();  // the LDS list is rebuilt for the next range
    if (P.gticks && threadIdx.x < kRangeWords && blk * kRangeWords + threadIdx.x < nwords)
      P.gticks[blk * kRangeWords + threadIdx.x] = wall_clock64();
  }
  flush_counters<FULL>(P, c);
  if (FULL == 2 && c_reads && P.counters)
    atomicAdd(P.counters + ACT_CNT_NODE_READS, (unsigned long long)c_reads);
}

// The second pass after a probe that listed its pending points per wave
// (kExactList): wave w of this kernel resolves the entries of probe wave w,
// one per lane, 64 at a time. The entry carries the point's code, so the
// lookup-table read can start beside the point's.
constexpr int kListBlock = 256;

// COUNT: a count join's resolve; its blocks keep a histogram of the
// polygons in LDS when the probe's did (hist_bins), so that the matches of
// pending points meet few global atomics; the grid then takes several probe
// waves' lists per wave.
template <int FULL, bool COUNT = false>
__global__ __launch_bounds__(kListBlock) void resolve_list_kernel(ProbeParams P,
                                                                  uint32_t nwaves) {
  extern __shared__ uint32_t s_counts[];
  uint32_t *s_hist = COUNT && P.hist_bins > 0 ? s_counts : nullptr;
  if (s_hist) {
    for (int k = threadIdx.x; k < P.hist_bins; k += kListBlock) s_hist[k] = 0u;
    __syncthreads();
  }
  const int lane = threadIdx.x & 63;
  uint32_t c[7] = {0, 0, 0, 0, 0, 0, 0}, c_reads = 0;
  const uint32_t stride = gridDim.x * (kListBlock / 64);
  for (uint32_t w = blockIdx.x * (kListBlock / 64) + (threadIdx.x >> 6); w < nwaves; w += stride) {
    const uint32_t cnt = P.pcount[w];
    const uint2 *list = P.plist + (size_t)w * P.region;
    for (uint32_t e = lane; e < cnt; e += 64) {
      const uint2 ent = list[e];
      resolve_point<FULL, false, false, COUNT>(P, ent.x, ent.y, c, c_reads, s_hist);
    }
  }
  if (s_hist) {
    __syncthreads();
    for (int k = threadIdx.x; k < P.hist_bins; k += kListBlock) {
      const uint32_t v = s_hist[k];
      if (v) atomicAdd(P.counts + k, (unsigned long long)v);
    }
  }
  flush_counters<FULL>(P, c);
  if (FULL == 2 && c_reads && P.counters)
    atomicAdd(P.counters + ACT_CNT_NODE_READS, (unsigned long long)c_reads);
}

// ------------------------------------------------------------------ probe

// Probe modes: approximate (every reference of a cell is a hit); exact,
// leaving pending points in a mask for resolve_kernel; exact, with pending
// points resolved by the probe's own waves (cell-local refinement); exact,
// with pending points listed per wave for resolve_list_kernel (cell-local
// refinement).
// Count joins (per-polygon number of covering points, no out[]) have modes
// of their own: approximate, and exact with per-wave pending lists.
enum ProbeMode {
  kApprox = 0,
  kExactMask = 1,
  kExactFused = 2,
  kExactList = 3,
  kApproxCount = 4,
  kExactCount = 5
};

// A wave's queue of pending points (kExactFused). The probe appends each
// finished tile's pending points; whenever 64 have gathered, the wave
// resolves them, one per lane, so refinement runs on full waves and needs no
// second pass over the points. Entries are ring slots (head + k) mod
// kQueueCap holding a point's index and its cell entry.
constexpr int kQueueCap = 256;

struct PendingQueue {
  int64_t *v;
  uint64_t *e;
  uint32_t head, count;  // wave-uniform
  uint2 *list;           // kExactList: this wave's region of the pending list
};

// Pair output of approximate joins goes through a per-block buffer in LDS:
// a wave reserves its pairs' slots there with one LDS atomic, and the block
// moves the buffer to the pair list with one global atomic when it ends
// (every wave reserving its own slots in the global list instead meets a
// single, heavily contended counter). A wave whose pairs do not fit writes
// them to the list directly and marks its slots in the buffer unused.
constexpr int kPairBuf = 1024;  // pairs (12 KiB), one per probe thread at the flush

struct PairBuf {
  int64_t *pt;
  int32_t *poly;
  uint32_t *count;  // slots reserved so far (may pass kPairBuf)
};

// Resolves the first n (<= 64) queued points, lane l taking entry l.
template <int FULL, bool BATCHED>
__device__ __forceinline__ void drain_queue(const ProbeParams &P, PendingQueue &Q, uint32_t n,
                                            int lane, uint32_t (&rc)[7], uint32_t &c_reads) {
  const bool on = (uint32_t)lane < n;
  int64_t v = 0;
  uint64_t e = 0;
  if (on) {
    const uint32_t slot = (Q.head + (uint32_t)lane) & (kQueueCap - 1);
    v = Q.v[slot];
    e = Q.e[slot];
  }
  wave_sync();  // read before later appends reuse the slots
  Q.head += n;
  Q.count -= n;
  if (on) resolve_point<FULL, BATCHED, true>(P, v, e, rc, c_reads);
}

// Step 7-9 for the NP points of a lane in tile `tile` (points at T).
template <int MODE, int FULL, int NP, bool BATCHED>
__device__ __forceinline__ void finish_tile(const ProbeParams &P, uint32_t tile, const TileRef &T,
                                            int lane, const uint32_t (&e)[NP],
                                            const bool (&live)[NP], const bool (&valid)[NP],
                                            uint32_t (&c)[8], PendingQueue &Q, uint32_t (&rc)[7],
                                            uint32_t &c_reads, uint32_t *s_hist,
                                            const PairBuf &PB) {
  bool pend[NP];
  const __amdgpu_buffer_rsrc_t out_buf = tile_buffer(T.out, 4 * T.n);
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const int k = p * 64 + lane;  // within the tile
    const int64_t i = T.gi + k;   // caller's index (pair output)
    if (FULL == 2) {
      c[0] += live[p];
      c[1] += live[p] && !valid[p];
      c[2] += valid[p] && e[p] == 0;
    }
    // stage 3: the entry's references (Section III-E: one payload, two
    // payloads or a lookup-table offset)
    // (32-bit entries: the builder narrows every two-reference entry whose
    // second reference is not 0, a candidate, to a lookup-table list)
    const uint32_t tag = e[p] & (uint32_t)kTagMask;
    const uint32_t r0 = e[p] >> 2;
    const uint32_t r1 = 0u;
    const int n_inl = e[p] == 0 || tag == kTagLut ? 0 : (tag == kTagTwo ? 2 : 1);
    const uint32_t off = e[p] >> 2;
    if (MODE == kApproxCount) {
      // approximate count join: every reference of the cell is a match
      if (live[p]) {
        if (n_inl > 0) count_add(P, s_hist, r0 >> 1);
        if (n_inl > 1) count_add(P, s_hist, r1 >> 1);
        if (tag == kTagLut) {
          const uint32_t nt = P.lut[off];
          for (uint32_t r = 0; r < nt; r++) count_add(P, s_hist, P.lut[off + 1 + r]);
          const uint32_t nc = P.lut[off + 1 + nt];
          for (uint32_t r = 0; r < nc; r++) count_add(P, s_hist, P.lut[off + 2 + nt + r]);
        }
      }
      pend[p] = false;
    } else if (MODE == kApprox) {
      // approximate mode: every reference is reported, the lowest in out[]
      Hits<false> hits;
      if (n_inl > 0) hits.add(P, i, (int32_t)(r0 >> 1));
      if (n_inl > 1) hits.add(P, i, (int32_t)(r1 >> 1));
      uint32_t nt = 0, nc = 0;
      if (tag == kTagLut) {
        nt = P.lut[off];
        nc = P.lut[off + 1 + nt];
        // each part of a list is sorted, so the lowest id heads a part
        // (the device copy of the table is padded: the reads stay in
        // bounds when a part is empty)
        const uint32_t t0 = P.lut[off + 1], c0 = P.lut[off + 2 + nt];
        if (nt) hits.add(P, i, (int32_t)t0);
        if (nc) hits.add(P, i, (int32_t)c0);
        if (FULL == 2) c[4]++;
      }
      if (FULL >= 1 && P.pair_pt) {
        // every other reference is a pair; the wave reserves the slots of
        // all its lanes' pairs in the block's buffer at once
        const uint32_t refs = live[p] ? (uint32_t)n_inl + nt + nc : 0u;
        const uint32_t k = refs > 0 ? refs - 1 : 0u;
        // (most waves have no pair beyond out[]: they skip the scan)
        if (ballot(k != 0u) != 0ull) {  // wave-uniform
          uint32_t incl = k;
#pragma unroll
          for (int d = 1; d < 64; d <<= 1) {
            const uint32_t v = __shfl_up(incl, d);
            if (lane >= d) incl += v;
          }
          const uint32_t total = __shfl(incl, 63);
          uint32_t lb = 0;
          if (lane == 0) lb = atomicAdd(PB.count, total);
          lb = __shfl(lb, 0);
          const bool fits = lb + total <= (uint32_t)kPairBuf;
          unsigned long long gb = 0;
          if (!fits) {
            if (lane == 0) gb = atomicAdd((unsigned long long *)P.n_pairs, (unsigned long long)total);
            gb = __shfl(gb, 0);
            for (uint32_t q = lb + lane; q < min(lb + total, (uint32_t)kPairBuf); q += 64)
              PB.poly[q] = -1;  // reserved but unused
          }
          uint32_t m = incl - k;
          auto put = [&](int32_t poly) {
            if (poly == hits.best) return;
            if (fits) {
              PB.pt[lb + m] = i;
              PB.poly[lb + m] = poly;
            } else if ((int64_t)(gb + m) < P.cap) {
              P.pair_pt[gb + m] = i;
              P.pair_poly[gb + m] = poly;
            }
            m++;
          };
          if (live[p]) {
            if (n_inl > 0) put((int32_t)(r0 >> 1));
            if (n_inl > 1) put((int32_t)(r1 >> 1));
            for (uint32_t r = 0; r < nt; r++) put((int32_t)P.lut[off + 1 + r]);
            for (uint32_t r = 0; r < nc; r++) put((int32_t)P.lut[off + 2 + nt + r]);
          }
        }
      }
      if (FULL == 2) c[3] += e[p] != 0;
      // every lane stores (past the tile's end the range check drops it),
      // so the store is always issued and the compiler's waits stay exact
      __builtin_amdgcn_raw_buffer_store_b32((uint32_t)hits.best, out_buf, 4 * k, 0, kBufferNT);
      pend[p] = false;
    } else {
      // exact mode: a point whose cell entry has candidate references or is
      // a lookup-table list is pending. Its list offset goes to out[]; then
      // either its bit goes to the pending mask (resolve_kernel finishes
      // it) or the point joins the wave's queue.
      // With 32-bit entries the only entry without candidates that has a
      // reference is a one-reference entry (tag 01) whose reference is
      // interior (bit 2): a two-reference entry's second reference is
      // candidate 0. So a live point is pending exactly when its entry is a
      // list, a two-reference entry or a one-reference entry with a
      // candidate, and a point that is not pending has at most one
      // (interior) reference: no pair beyond out[].
      (void)r1;
      const bool one_true = tag == kTagOne && (e[p] & 4u) != 0u;
      pend[p] = live[p] && (tag == kTagLut || tag == kTagTwo || (tag == kTagOne && !one_true));
      // the wave's pending lanes, taken once while the predicate is a mask
      const uint64_t pm = ballot(pend[p]);
      int32_t v;
      if (MODE == kExactCount) {
        if (live[p] && one_true) count_add(P, s_hist, e[p] >> 3);
        v = 0;
      } else {
        v = tag == kTagLut ? -3 - (int32_t)off
            : pend[p]      ? kPending
            : one_true     ? (int32_t)(e[p] >> 3)
                           : -1;
        if (FULL == 2) c[3] += !pend[p] && live[p] && e[p] != 0;
      }
      if (MODE == kExactFused && pend[p]) {
        const uint32_t slot = (Q.head + Q.count + (uint32_t)lane_rank(pm)) & (kQueueCap - 1);
        Q.v[slot] = (int64_t)tile * (64 * NP) + k;
        Q.e[slot] = e[p];
      }
      // one store from every lane (dropped past the tile's end); a count
      // join writes no out[]
      if (MODE != kExactCount)
        __builtin_amdgcn_raw_buffer_store_b32((uint32_t)v, out_buf, 4 * k, 0, kBufferNT);
      if (MODE == kExactFused) Q.count += (uint32_t)__popcll(pm);
      if (MODE == kExactList || MODE == kExactCount) {
        // the wave appends its pending points (index in the pass, code) to
        // its region of the list, through a buffer over the region's free
        // part: the other lanes' stores are out of range and dropped
        // (the region's free part, capped below the out-of-range offset:
        // it always holds the wave's next 64 entries)
        const __amdgpu_buffer_rsrc_t lb = tile_buffer(
            Q.list + Q.count,
            (int32_t)min<uint64_t>(8ull * (P.region - Q.count), (uint64_t)kBufferOutOfRange));
        const act_int2_v w = {(int)(tile * (uint32_t)(64 * NP) + (uint32_t)k), (int)v};
        __builtin_amdgcn_raw_buffer_store_b64(w, lb, pend[p] ? 8 * lane_rank(pm) : kBufferOutOfRange,
                                              0, 0);
        Q.count += (uint32_t)__popcll(pm);
      }
    }
  }
  if (MODE == kExactMask) {
#pragma unroll
    for (int p = 0; p < NP; p++) {
      const uint64_t m = ballot(pend[p]);
      // every lane stores the word (the same value), a word past the pass
      // to the sink; every group of a batched join's virtual space has one
      uint64_t *word = BATCHED || p * 64 < T.n ? P.mask + (int64_t)tile * NP + p : P.sink + 1;
      *word = m;
    }
  }
  if (MODE == kExactFused && Q.count >= 64) {
    wave_sync();  // appended before they are read
    do {
      drain_queue<FULL, BATCHED>(P, Q, 64, lane, rc, c_reads);
    } while (Q.count >= 64);
  }
  if (P.gticks && lane < NP) P.gticks[(int64_t)tile * NP + lane] = wall_clock64();
}

// Loads the points of tile T into v (lanes past its end read zeros, which
// they do not use). IDS: the tile's precomputed cell ids are loaded instead
// (8 bytes each, carried in the x half).
template <int NP, bool IDS = false>
__device__ __forceinline__ void load_tile(const TileRef &T, int lane, double2 (&v)[NP]) {
  const __amdgpu_buffer_rsrc_t buf =
      IDS ? tile_buffer(T.ids, 8 * T.n) : tile_buffer(T.pts, 16 * T.n);
#pragma unroll
  for (int p = 0; p < NP; p++) {
    const int k = p * 64 + lane;
    if (IDS) {
      const act_int2_v w = __builtin_amdgcn_raw_buffer_load_b64(buf, 8 * k, 0, kBufferNT);
      v[p] = make_double2(__hiloint2double(w.y, w.x), 0.0);
    } else {
      const act_int4_v w = __builtin_amdgcn_raw_buffer_load_b128(buf, 16 * k, 0, kBufferNT);
      v[p] = make_double2(__hiloint2double(w.y, w.x), __hiloint2double(w.w, w.z));
    }
  }
}

// Leaf coordinates of a level-30 cell id (face, 60-bit Hilbert position,
// marker bit): the position is read 4 levels (8 bits) at a time through the
// inverse of the curve's 4-level state table, from the two padding levels
// of the 32-level frame down. Ids of no leaf (face above 5, no marker at
// bit 0, including 0) are invalid.
__device__ __forceinline__ bool decode_leaf(const uint16_t *hinv, uint64_t id, uint32_t &face,
                                            uint32_t &i, uint32_t &j) {
  face = (uint32_t)(id >> 61);
  const uint64_t pos = (id >> 1) & ((1ull << 60) - 1);
  uint32_t st = 0, ii = 0, jj = 0;
#pragma unroll
  for (int sh = 56; sh >= 0; sh -= 8) {
    const uint32_t e = hinv[(st << 8) | (uint32_t)((pos >> sh) & 255u)];
    ii = (ii << 4) | ((e >> 4) & 15u);
    jj = (jj << 4) | (e & 15u);
    st = e >> 8;
  }
  i = ii;
  j = jj;
  return face <= 5u && (id & 1ull);
}

// Steps 2-5 and the LDS-staged part of step 6 for the points of tile T.
template <int LDS_DEPTH, int NP, bool IDS = false>
__device__ __forceinline__ void project_tile(const double2 *s_trig, const uint32_t *s_nodes,
                                             const FaceDev *s_face, const TileRef &T, int lane,
                                             const double2 (&pts)[NP], Descent<NP> &D,
                                             bool (&live)[NP], bool (&valid)[NP],
                                             uint32_t &c_reads, const uint16_t *s_hinv) {
  uint32_t face[NP], ci[NP], cj[NP];
#pragma unroll
  for (int p = 0; p < NP; p++) {
    live[p] = p * 64 + lane < T.n;
    face[p] = ci[p] = cj[p] = 0;
    if (IDS) {
      valid[p] = live[p] && decode_leaf(s_hinv, (uint64_t)__double_as_longlong(pts[p].x), face[p],
                                        ci[p], cj[p]);
      face[p] = valid[p] ? face[p] : 0u;
    } else {
      valid[p] = live[p] && project(s_trig, pts[p].x, pts[p].y, face[p], ci[p], cj[p]);
    }
  }
  descend_lds<LDS_DEPTH, NP>(s_nodes, s_face, face, ci, cj, valid, D, c_reads);
}

// The probe. Each wavefront walks tiles of 64 * NP consecutive points (NP
// per lane, at lane and lane + 64, ...), grid-stride, so all lanes of a
// wave run the same number of iterations. The loop is a two-stage software
// pipeline: while tile t is projected and descends the LDS-staged levels,
// the first global node level of tile t - 1 (issued at the end of the
// previous iteration) is in flight; then tile t - 1 finishes. The point
// loads run one tile further ahead.
// Waves per SIMD the compiler must make room for. Eight (two 1024-thread
// blocks per CU: at most 64 VGPRs and few SGPRs) where the probe fits
// without spilling in its loop; the probe that resolves its own queue keeps
// its registers (one block per CU).
template <int MODE, int NP>
constexpr int kProbeWavesPerEU = MODE != kExactFused ? 8 : 1;

// IDS: the points arrive as level-30 cell ids (Listing 3's input), decoded
// instead of projected.
template <int MODE, int LDS_DEPTH, int FULL, int NP, bool BATCHED, bool IDS = false>
__global__ __launch_bounds__(kProbeBlock, (kProbeWavesPerEU<MODE, NP>)) void probe_kernel(
    ProbeParams P) {
  constexpr bool FUSED = MODE == kExactFused;
  extern __shared__ uint32_t s_nodes[];
  __shared__ FaceDev s_face[6];
  __shared__ double2 s_trig[IDS ? 1 : kTrigEntries];
  __shared__ uint16_t s_hinv[IDS ? 1024 : 1];
  constexpr bool PAIRBUF = FULL >= 1 && MODE == kApprox;
  __shared__ int64_t s_ppt[PAIRBUF ? kPairBuf : 1];
  __shared__ int32_t s_ppo[PAIRBUF ? kPairBuf : 1];
  __shared__ uint32_t s_pcnt;
  __shared__ unsigned long long s_pbase;
  __shared__ uint32_t s_pwave[kProbeWaves];
  const PairBuf PB{s_ppt, s_ppo, &s_pcnt};
  __shared__ int64_t s_qv[FUSED ? kProbeWaves * kQueueCap : 1];
  __shared__ uint64_t s_qe[FUSED ? kProbeWaves * kQueueCap : 1];
  if (LDS_DEPTH > 0)
    for (int k = threadIdx.x; k < P.n_lds_nodes * 256; k += kProbeBlock) s_nodes[k] = P.top32[k];
  if (threadIdx.x < 6) s_face[threadIdx.x] = P.faces[threadIdx.x];
  if (!IDS && threadIdx.x < kTrigEntries) s_trig[threadIdx.x] = P.trig[threadIdx.x];
  if (IDS) s_hinv[threadIdx.x] = P.hinv[threadIdx.x];  // 1024 threads, 1024 entries
  if (PAIRBUF && threadIdx.x == 0) s_pcnt = 0;
  // count joins: a per-block histogram of the polygons after the trie levels
  constexpr bool COUNTING = MODE == kApproxCount || MODE == kExactCount;
  uint32_t *s_hist = COUNTING && P.hist_bins > 0 ? s_nodes + P.n_lds_nodes * 256 : nullptr;
  if (s_hist)
    for (int k = threadIdx.x; k < P.hist_bins; k += kProbeBlock) s_hist[k] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wid = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave-uniform
  uint32_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0}, c_reads = 0;
  uint32_t rc[7] = {0, 0, 0, 0, 0, 0, 0};  // resolve counters (kExactFused)
  PendingQueue Q{s_qv + (FUSED ? wid * kQueueCap : 0), s_qe + (FUSED ? wid * kQueueCap : 0), 0u, 0u,
                 MODE == kExactList || MODE == kExactCount
                     ? P.plist + (size_t)(blockIdx.x * kProbeWaves + wid) * P.region
                     : nullptr};
  constexpr int TILE = 64 * NP;
  const uint32_t ntiles = (uint32_t)(BATCHED ? P.vhdr[0] / NP : (P.n + TILE - 1) / TILE);
  const uint32_t nwaves = gridDim.x * kProbeWaves;
  const uint32_t first = blockIdx.x * kProbeWaves + wid;
  if (first < ntiles) {
    // stage B: the tile whose first global level is in flight; nxt: the
    // points of the tile after the one being projected
    Descent<NP> B;
    uint32_t xB[NP];
    bool liveB[NP], validB[NP];
    TileRef TB = tile_ref<BATCHED, NP>(P, first), TN;
    uint32_t tileB = first;
    double2 nxt[NP];
    {  // prologue: the wave's first tile
      double2 cur[NP];
      load_tile<NP, IDS>(TB, lane, cur);
      TN = first + nwaves < ntiles ? tile_ref<BATCHED, NP>(P, first + nwaves) : TB;
      load_tile<NP, IDS>(TN, lane, nxt);
      project_tile<LDS_DEPTH, NP, IDS>(s_trig, s_nodes, s_face, TB, lane, cur, B, liveB, validB,
                                       c_reads, s_hinv);
      issue_level<NP, LDS_DEPTH>(P, B, xB);
    }
    // steady state: no wave-uniform branches around memory operations, so
    // the compiler's waits for the node level in flight and for the next
    // tile's points stay exact
    for (uint32_t tile = first + nwaves; tile < ntiles; tile += nwaves) {
      const TileRef TA = TN;
      TN = tile + nwaves < ntiles ? tile_ref<BATCHED, NP>(P, tile + nwaves) : TA;
      double2 cur[NP];
#pragma unroll
      for (int p = 0; p < NP; p++) cur[p] = nxt[p];
      load_tile<NP, IDS>(TN, lane, nxt);
      Descent<NP> A;
      bool liveA[NP], validA[NP];
      project_tile<LDS_DEPTH, NP, IDS>(s_trig, s_nodes, s_face, TA, lane, cur, A, liveA, validA,
                                       c_reads, s_hinv);
      take_level<NP>(B, xB, c_reads);
      descend_rest<NP, LDS_DEPTH + 1>(P, B, c_reads);
      finish_tile<MODE, FULL, NP, BATCHED>(P, tileB, TB, lane, B.e, liveB, validB, c, Q, rc,
                                            c_reads, s_hist, PB);
      B = A;
      TB = TA;
      tileB = tile;
#pragma unroll
      for (int p = 0; p < NP; p++) {
        liveB[p] = liveA[p];
        validB[p] = validA[p];
      }
      issue_level<NP, LDS_DEPTH>(P, B, xB);
    }
    // epilogue: the wave's last tile
    take_level<NP>(B, xB, c_reads);
    descend_rest<NP, LDS_DEPTH + 1>(P, B, c_reads);
    finish_tile<MODE, FULL, NP, BATCHED>(P, tileB, TB, lane, B.e, liveB, validB, c, Q, rc,
                                          c_reads, s_hist, PB);
  }
  if (MODE == kExactList || MODE == kExactCount)
    P.pcount[blockIdx.x * kProbeWaves + wid] = Q.count;
  if (PAIRBUF && P.pair_pt) {
    // move the block's buffered pairs to the pair list: slots in use
    // (unused ones are marked), compacted with one global reservation
    __syncthreads();
    const uint32_t t = threadIdx.x;  // one slot per thread (kPairBuf = block size)
    const bool use = t < min(s_pcnt, (uint32_t)kPairBuf) && s_ppo[t] >= 0;
    const uint64_t bal = ballot(use);
    const uint32_t rank = (uint32_t)lane_rank(bal);
    if (lane == 0) s_pwave[wid] = (uint32_t)__popcll(bal);
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kProbeWaves; w++) {
      before += w < wid ? s_pwave[w] : 0u;
      all += s_pwave[w];
    }
    if (t == 0 && all)
      s_pbase = atomicAdd((unsigned long long *)P.n_pairs, (unsigned long long)all);
    __syncthreads();
    if (use) {
      const int64_t slot = (int64_t)(s_pbase + before + rank);
      if (slot < P.cap) {
        P.pair_pt[slot] = s_ppt[t];
        P.pair_poly[slot] = s_ppo[t];
      }
    }
  }
  if (s_hist) {
    __syncthreads();
    for (int k = threadIdx.x; k < P.hist_bins; k += kProbeBlock) {
      const uint32_t v = s_hist[k];
      if (v) atomicAdd(P.counts + k, (unsigned long long)v);
    }
  }
  if (FUSED && Q.count > 0) {
    wave_sync();
    drain_queue<FULL, BATCHED>(P, Q, Q.count, lane, rc, c_reads);
  }
  if (FUSED) flush_counters<FULL>(P, rc);
  if (FULL == 2 && P.counters) {
    unsigned long long *C = P.counters;
    atomicAdd(C + ACT_CNT_POINTS, (unsigned long long)c[0]);
    atomicAdd(C + ACT_CNT_INVALID, (unsigned long long)c[1]);
    atomicAdd(C + ACT_CNT_FALSE_HIT, (unsigned long long)c[2]);
    atomicAdd(C + ACT_CNT_SOLELY_TRUE, (unsigned long long)c[3]);
    atomicAdd(C + ACT_CNT_NODE_READS, (unsigned long long)c_reads);
    atomicAdd(C + ACT_CNT_LUT_READS, (unsigned long long)c[4]);
  }
}

// ---------------------------------------------------------------- batches
//
// A batched join lays its batches end to end in a virtual point space,
// each starting at a multiple of 128 points (so no probe tile spans two
// batches), and runs the probe and resolve kernels over that space once.
// The probe walks the space in order, so a batch's completion time grows
// with the points laid out before it: the batches are laid out smallest
// first, by size class (the bit length of the batch's 128-point blocks;
// input order within a class), which lets the many small batches of an
// uneven mix complete early without delaying the total. The setup kernel
// (one block) computes the layout; the fill kernel records the batch of
// every 64-point group; the finish kernel turns the groups' completion
// ticks into per-batch completion ticks. None of them needs the host to
// know the sizes, so the whole call can be captured.
constexpr int kSetupBlock = 1024;
constexpr int kSizeClasses = 40;  // bit lengths of 128-point block counts (< 2^37 points)

__device__ __forceinline__ int64_t batch_span(int64_t n) { return n > 0 ? (n + 127) / 128 * 128 : 0; }

__device__ __forceinline__ int size_class(int64_t span) {
  return span > 0 ? 64 - __clzll((unsigned long long)(span / 128)) : 0;
}

__global__ __launch_bounds__(kSetupBlock) void batch_setup_kernel(const act_batch *batches,
                                                                  int32_t nb, int64_t cap_groups,
                                                                  int64_t *vstart, int64_t *vsorted,
                                                                  int32_t *vorder, int64_t *vhdr,
                                                                  uint64_t *ticks) {
  __shared__ unsigned long long s_cls_pts[kSizeClasses];
  __shared__ unsigned int s_cls_cnt[kSizeClasses];
  __shared__ int64_t s_part[kSetupBlock / 64];
  __shared__ int32_t s_cpart[kSetupBlock / 64];
  __shared__ int64_t s_carry;
  __shared__ int32_t s_ccarry;
  if (threadIdx.x < kSizeClasses) {
    s_cls_pts[threadIdx.x] = 0;
    s_cls_cnt[threadIdx.x] = 0;
  }
  if (threadIdx.x == 0 && ticks) ticks[0] = wall_clock64();
  __syncthreads();
  // points and batches per size class
  bool bad = false;
  for (int32_t b = threadIdx.x; b < nb; b += kSetupBlock) {
    const int64_t n = batches[b].n;
    bad |= n < 0 || n >= (1ll << 37);
    const int64_t sp = (n < 0 || n >= (1ll << 37)) ? 0 : batch_span(n);
    const int c = size_class(sp);
    atomicAdd(&s_cls_pts[c], (unsigned long long)sp);
    atomicAdd(&s_cls_cnt[c], 1u);
  }
  bad = __syncthreads_or(bad);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int64_t vbase = 0;
  int32_t cbase = 0;
  // each class in turn: an exclusive scan of its batches' spans (and
  // counts), in input order, from the class's first virtual point (and
  // first position of the order)
  for (int c = 0; c < kSizeClasses; c++) {
    const int64_t cls_pts = (int64_t)s_cls_pts[c];
    const int32_t cls_cnt = (int32_t)s_cls_cnt[c];
    if (cls_cnt == 0) continue;  // block-uniform
    if (threadIdx.x == 0) {
      s_carry = 0;
      s_ccarry = 0;
    }
    __syncthreads();
    for (int32_t b0 = 0; b0 < nb; b0 += kSetupBlock) {
      const int32_t b = b0 + (int32_t)threadIdx.x;
      int64_t sp = 0;
      int32_t one = 0;
      if (b < nb) {
        const int64_t n = batches[b].n;
        const int64_t s0 = (n < 0 || n >= (1ll << 37)) ? 0 : batch_span(n);
        if (size_class(s0) == c) {
          sp = s0;
          one = 1;
        }
      }
      int64_t incl = sp;
      int32_t cincl = one;
#pragma unroll
      for (int d = 1; d < 64; d <<= 1) {
        const int64_t v = __shfl_up(incl, d);
        const int32_t w = __shfl_up(cincl, d);
        if (lane >= d) {
          incl += v;
          cincl += w;
        }
      }
      if (lane == 63) {
        s_part[wid] = incl;
        s_cpart[wid] = cincl;
      }
      __syncthreads();
      int64_t before = s_carry, total = 0;
      int32_t cbefore = s_ccarry, ctotal = 0;
      for (int k = 0; k < kSetupBlock / 64; k++) {
        if (k < wid) {
          before += s_part[k];
          cbefore += s_cpart[k];
        }
        total += s_part[k];
        ctotal += s_cpart[k];
      }
      if (one) {
        const int64_t v = vbase + before + incl - sp;
        const int32_t pos = cbase + cbefore + cincl - 1;
        vstart[b] = v;
        vsorted[pos] = v;
        vorder[pos] = b;
      }
      __syncthreads();
      if (threadIdx.x == 0) {
        s_carry += total;
        s_ccarry += ctotal;
      }
      __syncthreads();
    }
    vbase += cls_pts;
    cbase += cls_cnt;
  }
  if (threadIdx.x == 0) {
    vstart[nb] = vbase;
    vsorted[nb] = vbase;
    const int64_t groups = vbase / 64;
    vhdr[0] = (bad || groups > cap_groups) ? 0 : groups;  // 0: the join does nothing
    vhdr[1] = (bad || groups > cap_groups) ? 1 : 0;
  }
}

__global__ __launch_bounds__(256) void batch_fill_kernel(const int64_t *vsorted,
                                                         const int32_t *vorder, int32_t nb,
                                                         const int64_t *vhdr,
                                                         int32_t *group_batch) {
  const int64_t ng = vhdr[0];
  for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < ng;
       g += (int64_t)gridDim.x * 256) {
    // the last batch in virtual order whose first point is at or before the
    // group's (empty batches, all of class 0, come first)
    int32_t lo = 0, hi = nb - 1;
    const int64_t v = g * 64;
    while (lo < hi) {
      const int32_t mid = (lo + hi + 1) >> 1;
      if (vsorted[mid] <= v) lo = mid; else hi = mid - 1;
    }
    group_batch[g] = vorder[lo];
  }
}

// Completion tick of each batch: the latest tick of its groups (the resolve
// kernel's, in exact mode, which runs after the probe).
__global__ __launch_bounds__(256) void batch_finish_kernel(const act_batch *batches,
                                                           const int64_t *vstart, int32_t nb,
                                                           const int64_t *vhdr,
                                                           const uint64_t *gticks,
                                                           uint64_t *ticks) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * 4;
  const bool ok = vhdr[0] > 0 || vstart[nb] == 0;
  for (int64_t b = wave; b < nb; b += nwaves) {
    uint64_t t = 0;
    if (ok) {
      const int64_t g0 = vstart[b] / 64, g1 = g0 + batch_span(batches[b].n) / 64;
      for (int64_t g = g0 + lane; g < g1; g += 64) t = max(t, gticks[g]);
    }
    for (int d = 32; d > 0; d >>= 1) t = max(t, (uint64_t)__shfl_xor(t, d));
    if (lane == 0) ticks[1 + b] = ok ? (t ? t : ticks[0]) : 0;
  }
}

__global__ __launch_bounds__(256) void cell_id_kernel(const double2 *pts, int64_t n,
                                                      const uint16_t *htab, const double2 *trig,
                                                      uint64_t *ids) {
  __shared__ uint16_t s_htab[1024];
  __shared__ double2 s_trig[kTrigEntries];
  for (int k = threadIdx.x; k < 1024; k += blockDim.x) s_htab[k] = htab[k];
  for (int k = threadIdx.x; k < kTrigEntries; k += blockDim.x) s_trig[k] = trig[k];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double2 p = pts[i];
    uint32_t face, ci, cj;
    ids[i] = project<true>(s_trig, p.x, p.y, face, ci, cj)
                 ? (((uint64_t)face << 61) | (hilbert60(s_htab, ci, cj) << 1) | 1ull)
                 : 0ull;
  }
}

// ============================================== host side: launches and the C ABI

using ProbeFn = void (*)(ProbeParams);
template <int MODE, int LDS, int FULL>
static ProbeFn probe_np(int np) {
  return np == 1 ? probe_kernel<MODE, LDS, FULL, 1, false> : probe_kernel<MODE, LDS, FULL, 2, false>;
}

template <int MODE>
// full: 0 = lean, 1 = pair output, 2 = pair output and counters
static ProbeFn probe_mode_fn(int lds_depth, int full, int np) {
  using F = ProbeFn (*)(int);
  static const F tab[3][3] = {
      {probe_np<MODE, 0, 0>, probe_np<MODE, 0, 1>, probe_np<MODE, 0, 2>},
      {probe_np<MODE, 1, 0>, probe_np<MODE, 1, 1>, probe_np<MODE, 1, 2>},
      {probe_np<MODE, 2, 0>, probe_np<MODE, 2, 1>, probe_np<MODE, 2, 2>}};
  return tab[lds_depth][full](np);
}

static ProbeFn probe_fn(int mode, int lds_depth, int count, int np) {
  return mode == kApprox      ? probe_mode_fn<kApprox>(lds_depth, count, np)
         : mode == kExactMask ? probe_mode_fn<kExactMask>(lds_depth, count, np)
         : mode == kExactList ? probe_mode_fn<kExactList>(lds_depth, count, np)
                              : probe_mode_fn<kExactFused>(lds_depth, count, np);
}

// Count joins: lean kernels only.
template <int MODE, int LDS>
static ProbeFn probe_count_np(int np) {
  return np == 1 ? probe_kernel<MODE, LDS, 0, 1, false> : probe_kernel<MODE, LDS, 0, 2, false>;
}

static ProbeFn probe_count_fn(bool exact, int lds_depth, int np) {
  using F = ProbeFn (*)(int);
  static const F tab[2][3] = {
      {probe_count_np<kApproxCount, 0>, probe_count_np<kApproxCount, 1>,
       probe_count_np<kApproxCount, 2>},
      {probe_count_np<kExactCount, 0>, probe_count_np<kExactCount, 1>,
       probe_count_np<kExactCount, 2>}};
  return tab[exact ? 1 : 0][lds_depth](np);
}

// Joins of precomputed cell ids: lean kernels, approximate or with the
// per-wave pending lists.
template <int MODE, int LDS>
static ProbeFn probe_ids_np(int np) {
  return np == 1 ? probe_kernel<MODE, LDS, 0, 1, false, true>
                 : probe_kernel<MODE, LDS, 0, 2, false, true>;
}

static ProbeFn probe_ids_fn(bool exact, int lds_depth, int np) {
  using F = ProbeFn (*)(int);
  static const F tab[2][3] = {
      {probe_ids_np<kApprox, 0>, probe_ids_np<kApprox, 1>, probe_ids_np<kApprox, 2>},
      {probe_ids_np<kExactList, 0>, probe_ids_np<kExactList, 1>, probe_ids_np<kExactList, 2>}};
  return tab[exact ? 1 : 0][lds_depth](np);
}

// Batched joins: no counters.
template <int MODE, int LDS>
static ProbeFn probe_batched_np(int np) {
  return np == 1 ? probe_kernel<MODE, LDS, 0, 1, true> : probe_kernel<MODE, LDS, 0, 2, true>;
}

static ProbeFn probe_batched_fn(int mode, int lds_depth, int np) {
  using F = ProbeFn (*)(int);
  static const F tab[3][3] = {
      {probe_batched_np<kApprox, 0>, probe_batched_np<kApprox, 1>, probe_batched_np<kApprox, 2>},
      {probe_batched_np<kExactMask, 0>, probe_batched_np<kExactMask, 1>,
       probe_batched_np<kExactMask, 2>},
      {probe_batched_np<kExactFused, 0>, probe_batched_np<kExactFused, 1>,
       probe_batched_np<kExactFused, 2>}};
  return tab[mode][lds_depth](np);
}

// ------------------------------------------------------------------ host

static int device_count() {
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) return 0;
  return n;
}

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (dev >= 0 && dev != prev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0) (void)hipSetDevice(prev);
  }
};

static void free_image(DevImage &d) {
  void *ptrs[] = {d.nodes, d.lut,   d.eoff,  d.origin, d.pm,   d.e32,
                  d.e64,   d.trig,  d.faces, d.sink,  d.hinv, d.normals};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  d = DevImage();
}

template <typename T>
static int upload(T *&dst, const void *src, size_t bytes, size_t &total) {
  size_t nb = std::max<size_t>(bytes, 16);
  hipError_t e = hipMalloc((void **)&dst, nb);
  if (e != hipSuccess) {
    dst = nullptr;
    return fail(ACT_E_OOM, std::string("hipMalloc: ") + hipGetErrorString(e));
  }
  total += nb;
  if (bytes) {
    e = hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) return fail(ACT_E_HIP, std::string("hipMemcpy: ") + hipGetErrorString(e));
  }
  return ACT_OK;
}

static void free_batch_workspace(Workspace &w) {
  void *ptrs[] = {w.bmask, w.gticks, w.group_batch, w.vstart, w.vhdr, w.vsorted, w.vorder};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  w.bmask = w.gticks = nullptr;
  w.group_batch = nullptr;
  w.vstart = w.vhdr = w.vsorted = nullptr;
  w.vorder = nullptr;
  w.cap_groups = 0;
  w.cap_batches = 0;
}

static void free_workspace(Workspace &w) {
  if (w.mask) (void)hipFree(w.mask);
  if (w.plist) (void)hipFree(w.plist);
  if (w.pcount) (void)hipFree(w.pcount);
  free_batch_workspace(w);
  w = Workspace();
}

// The stream's batched-join buffers for nb batches of `points` points in
// total; allocated or enlarged when too small (not allowed while the stream
// is being captured). Call with the index's device current.
static int get_batch_workspace(const act_index *x, void *stream, int32_t nb, int64_t points,
                               Workspace *&out) {
  std::lock_guard<std::mutex> lk(x->ws_mu);
  Workspace &w = x->ws[stream];
  const int64_t groups = (points + 128 * (int64_t)nb) / 64 + 2;
  if (groups * 64 > kMaxLaunchPoints)
    return fail(ACT_E_RANGE, "batched join larger than 2^37 points (with padding)");
  if (w.cap_groups < groups || w.cap_batches < nb) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess &&
        cs != hipStreamCaptureStatusNone)
      return fail(ACT_E_RANGE, "batched workspace too small during stream capture; call "
                               "act_batched_reserve first");
    if (w.cap_groups && hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
      return fail(ACT_E_HIP, "cannot synchronise the stream to enlarge its workspace");
    const int64_t g = std::max(groups, w.cap_groups);
    const int32_t b = std::max(nb, w.cap_batches);
    free_batch_workspace(w);
    bool ok = hipMalloc((void **)&w.bmask, 8 * (size_t)g) == hipSuccess &&
              hipMalloc((void **)&w.gticks, 8 * (size_t)g) == hipSuccess &&
              hipMalloc((void **)&w.group_batch, 4 * (size_t)g) == hipSuccess &&
              hipMalloc((void **)&w.vstart, 8 * ((size_t)b + 1)) == hipSuccess &&
              hipMalloc((void **)&w.vsorted, 8 * ((size_t)b + 1)) == hipSuccess &&
              hipMalloc((void **)&w.vorder, 4 * ((size_t)b + 1)) == hipSuccess &&
              hipMalloc((void **)&w.vhdr, 64) == hipSuccess;
    if (!ok) {
      free_batch_workspace(w);
      return fail(ACT_E_OOM, "cannot allocate the batched-join workspace");
    }
    w.cap_groups = g;
    w.cap_batches = b;
  }
  out = &w;
  return ACT_OK;
}

// The stream's workspace: allocated on first use for `cap` points (and
// enlarged only when `grow` is set). Call with the index's device current.
// The mask needs no clearing: every pass writes each word it reads.
static int get_workspace(const act_index *x, void *stream, int64_t cap, bool grow,
                         Workspace *&out) {
  std::lock_guard<std::mutex> lk(x->ws_mu);
  Workspace &w = x->ws[stream];
  if (w.cap == 0 || (grow && w.cap < cap)) {
    cap = (cap + 63) / 64 * 64;
    if (w.mask && hipStreamSynchronize((hipStream_t)stream) != hipSuccess)
      return fail(ACT_E_HIP, "cannot synchronise the stream to enlarge its workspace");
    free_workspace(w);
    const int64_t plist_cap = cap + kListWavesMax * 128;
    if (hipMalloc((void **)&w.mask, (size_t)cap / 8) != hipSuccess ||
        hipMalloc((void **)&w.plist, 8 * (size_t)plist_cap) != hipSuccess ||
        hipMalloc((void **)&w.pcount, 4 * (size_t)kListWavesMax) != hipSuccess) {
      free_workspace(w);
      return fail(ACT_E_OOM, "cannot allocate the pending workspace");
    }
    w.cap = cap;
    w.plist_cap = plist_cap;
  }
  out = &w;
  return ACT_OK;
}

// ------------------------------------------------ joins that allocate nothing
//
// act_join_noalloc keeps the pending mask of its exact joins (one bit per
// point) in this file-scope device array instead of a per-stream workspace.
// Every device the library runs on holds its own copy for the life of the
// process. In host code the array's name is not a device address: the
// address is looked up once per device, with that device current, and only
// that pointer is handed to kernels. The mask needs no clearing: every probe
// writes each mask word its resolve kernel reads.
constexpr int64_t kNoAllocMaxPoints = 1ll << 27;  // points per call (16 MiB of mask)
static __device__ __align__(256) uint64_t scratch[kNoAllocMaxPoints / 64];

constexpr int kMaxDevices = 64;

static int noalloc_scratch(int dev, uint64_t *&ptr) {
  static std::mutex mu;
  static uint64_t *ptrs[kMaxDevices] = {nullptr};
  if (dev < 0 || dev >= kMaxDevices) return fail(ACT_E_DEVICE, "device index out of range");
  std::lock_guard<std::mutex> lk(mu);
  if (!ptrs[dev]) {
    DeviceGuard g(dev);
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ACT_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    ptrs[dev] = (uint64_t *)p;
  }
  ptr = ptrs[dev];
  return ACT_OK;
}

static void face_table(const HostIndex &h, FaceDev f[6]) {
  for (int k = 0; k < 6; k++) {
    const FaceRoot &F = h.faces[k];
    f[k] = FaceDev{F.root, kMaxLevel - F.plevel, F.pi, F.pj};
  }
}

// (cos b, sin b) for whole degrees b = -180 .. 180, by the C library.
static void trig_table(std::vector<double2> &t) {
  t.resize(kTrigEntries);
  for (int b = -180; b <= 180; b++) {
    const double a = b * (M_PI / 180.0);
    t[b + 180] = make_double2(std::cos(a), std::sin(a));
  }
}

static int upload_image(act_index *x) {
  const HostIndex &h = x->host;
  DevImage &d = x->dev;
  std::vector<double2> trig;
  trig_table(trig);
  int rc;
  {  // the trie with 32-bit entries (the builder narrowed every entry)
    std::vector<uint32_t> n32(h.nodes.size());
    for (size_t k = 0; k < n32.size(); k++) n32[k] = (uint32_t)h.nodes[k];
    if ((rc = upload(d.nodes, n32.data(), n32.size() * 4, d.bytes))) return rc;
  }
  // the device copy of the lookup table (with the records) carries zero
  // padding: lut_refs reads a list's first four words together, and the
  // approximate probe reads the head of a list's candidate part even when
  // that part is empty, so reads near the table's end stay in bounds
  std::vector<uint32_t> lut(h.lut);
  lut.resize(lut.size() + 10, 0u);
  if ((rc = upload(d.lut, lut.data(), lut.size() * 4, d.bytes))) return rc;
  if ((rc = upload(d.eoff, h.poly_edge_off.data(), h.poly_edge_off.size() * 4, d.bytes))) return rc;
  if ((rc = upload(d.origin, h.poly_origin.data(), h.poly_origin.size() * 8, d.bytes))) return rc;
  if ((rc = upload(d.pm, h.poly_m.data(), h.poly_m.size() * 4, d.bytes))) return rc;
  if ((rc = upload(d.e32, h.edges32.data(), h.edges32.size() * 4, d.bytes))) return rc;
  if ((rc = upload(d.e64, h.edges64.data(), h.edges64.size() * 8, d.bytes))) return rc;
  if ((rc = upload(d.trig, trig.data(), trig.size() * sizeof(double2), d.bytes))) return rc;
  FaceDev f[6];
  face_table(h, f);
  if ((rc = upload(d.faces, f, sizeof f, d.bytes))) return rc;
  const uint64_t zeros[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  if ((rc = upload(d.sink, zeros, sizeof zeros, d.bytes))) return rc;
  // the inverse of the 4-level Hilbert table: (state, 8 position bits) ->
  // (i nibble << 4 | j nibble) | next state << 8
  uint16_t fwd[1024], inv[1024];
  hilbert_table4(fwd);
  for (int st = 0; st < 4; st++)
    for (int b = 0; b < 256; b++) {
      const uint16_t e = fwd[st * 256 + b];
      inv[st * 256 + (e & 255)] = (uint16_t)(b | (e & 0x300));
    }
  if ((rc = upload(d.hinv, inv, sizeof inv, d.bytes))) return rc;
  if (h.geometry == ACT_GEOM_SPHERE &&
      (rc = upload(d.normals, h.normals.data(), h.normals.size() * 8, d.bytes)))
    return rc;
  return ACT_OK;
}

static int check_stream_device(const act_index *x, void *stream) {
  int dev = -1;
  if (stream) {
    if (hipStreamGetDevice((hipStream_t)stream, &dev) != hipSuccess)
      return fail(ACT_E_ARG, "invalid stream");
  } else if (hipGetDevice(&dev) != hipSuccess) {
    return fail(ACT_E_DEVICE, "no current HIP device");
  }
  if (dev != x->device)
    return fail(ACT_E_DEVICE, "stream is on device " + std::to_string(dev) +
                                  ", index on device " + std::to_string(x->device));
  return ACT_OK;
}

static int grid_for(int64_t n, int block) {
  int64_t blocks = (n + block - 1) / block;
  return (int)std::min<int64_t>(std::max<int64_t>(blocks, 1), 8192);
}


// Node count staged in LDS for `depth` levels (0 if it does not fit).
static int lds_nodes_for(const HostIndex &h, int depth) {
  int n = depth >= 2 ? h.n_d0 + h.n_d1 : (depth == 1 ? h.n_d0 : 0);
  return n <= kLdsTrieNodes ? n : -1;
}

static int default_lds_depth(const HostIndex &h) {
  for (int d = 2; d >= 1; d--)
    if (lds_nodes_for(h, d) > 0) return d;
  return 0;
}

// The index's device image in the kernel parameters.
static void index_params(const act_index *x, int refine, int n_lds, ProbeParams &P) {
  P.nodes = x->dev.nodes;
  const uint64_t nb = 4ull * x->host.nodes.size();
  P.node_bytes32 = nb <= kNodeBuffer32Max ? (uint32_t)nb : 0u;
  P.lut = x->dev.lut;
  P.eoff = x->dev.eoff;
  P.origin = x->dev.origin;
  P.pm = x->dev.pm;
  P.e32 = x->dev.e32;
  P.e64 = x->dev.e64;
  P.trig = x->dev.trig;
  P.faces = x->dev.faces;
  P.top32 = x->dev.nodes + 256;  // node 1 onward: the top levels come first
  P.n_lds_nodes = n_lds;
  P.refine = refine == ACT_REFINE_AUTO ? ACT_REFINE_LOCAL : refine;
  // records live in the LUT (planar exact indexes; spherical ones have none)
  P.local = x->host.mode == ACT_EXACT && x->host.geometry == ACT_GEOM_PLANE ? x->dev.lut : nullptr;
  P.normals = x->host.geometry == ACT_GEOM_SPHERE ? x->dev.normals : nullptr;
  P.sink = x->dev.sink;
  P.hinv = x->dev.hinv;
}

// Points per probe lane when a join leaves it to the index.
static int launch_np(const act_index *x) { return x->launch.points_per_lane; }

// `ext`: a caller-provided pending workspace (its mask only; cap points per
// pass) used instead of the stream's, so that the join allocates nothing.
// `counts`: a count join (per-polygon number of covering points added to
// counts[], no out[]); always with cell-local refinement and, in exact mode,
// the per-wave pending lists.
constexpr int64_t kCountPass = 1ll << 31;  // points per pass of a count join
constexpr int kCountGridMax = 4096;        // so that the pending lists always fit
constexpr int kLdsDynamicMax = 65536;      // dynamic LDS per probe block

// `ids`: the points' level-30 cell ids (a->d_points then only for pending
// points of exact joins, which use the per-wave lists).
static int join_impl(const act_index *x, const act_join_args *a, void *stream,
                     Workspace *ext = nullptr, unsigned long long *counts = nullptr,
                     const uint64_t *ids = nullptr) {
  if (!x) return fail(ACT_E_ARG, "index is NULL");
  if (!a) return fail(ACT_E_ARG, "args is NULL");
  if (a->n < 0) return fail(ACT_E_ARG, "n < 0");
  if (x->device < 0) return fail(ACT_E_DEVICE, "index was built without a device");
  if (a->n > 0 && (!a->d_out && !counts)) return fail(ACT_E_ARG, "out is NULL");
  if (a->n > 0 && !a->d_points && !(ids && x->host.mode == ACT_APPROX))
    return fail(ACT_E_ARG, "points is NULL");
  bool pairs = a->d_pair_point || a->d_pair_poly || a->d_n_pairs;
  if (pairs && (!a->d_pair_point || !a->d_pair_poly || !a->d_n_pairs || a->pair_capacity < 0))
    return fail(ACT_E_ARG, "pair output needs point, poly, counter arrays and capacity >= 0");
  if (a->refine < ACT_REFINE_AUTO || a->refine > ACT_REFINE_FP64)
    return fail(ACT_E_ARG, "unknown refine mode");
  if (a->block != 0 && a->block != kProbeBlock) return fail(ACT_E_ARG, "block must be 0 or 1024");
  if (a->grid < 0 || a->grid > 65536) return fail(ACT_E_ARG, "grid must be 0 .. 65536");
  if (a->pass_points < 0) return fail(ACT_E_ARG, "pass_points < 0");
  if (a->points_per_lane < 0 || a->points_per_lane > 2)
    return fail(ACT_E_ARG, "points_per_lane must be 0, 1 or 2");
  if (a->pending < ACT_PENDING_AUTO || a->pending > ACT_PENDING_QUEUE)
    return fail(ACT_E_ARG, "unknown pending mode");
  const HostIndex &h = x->host;
  const act_launch &L = x->launch;
  const int lds_req = a->lds_levels >= 0 ? a->lds_levels : L.lds_levels;
  int depth = lds_req < 0 ? default_lds_depth(h) : lds_req;
  if (depth > 2) return fail(ACT_E_ARG, "lds_levels must be -1, 0, 1 or 2");
  int n_lds = depth > 0 ? lds_nodes_for(h, depth) : 0;
  if (n_lds < 0) return fail(ACT_E_RANGE, "top trie levels do not fit the LDS budget");
  if (depth > 0 && n_lds == 0) depth = 0;  // empty trie
  int rc = check_stream_device(x, stream);
  if (rc) return rc;
  if (a->n == 0) return ACT_OK;
  ProbeParams P{};
  P.pts = (const double2 *)a->d_points;
  P.n = a->n;
  P.out = a->d_out;
  P.pair_pt = pairs ? a->d_pair_point : nullptr;
  P.pair_poly = a->d_pair_poly;
  P.cap = a->pair_capacity;
  P.n_pairs = a->d_n_pairs;
  P.counters = (unsigned long long *)a->d_counters;
  index_params(x, a->refine == ACT_REFINE_AUTO ? L.refine : a->refine, n_lds, P);
  const int np = a->points_per_lane > 0 ? a->points_per_lane : launch_np(x);
  DeviceGuard g(x->device);
  const bool exact = h.mode == ACT_EXACT;
  // counters or pair output: the full kernels (plain joins run lean ones)
  // 0: lean kernels, 1: pair output, 2: pair output and counters
  const int count = a->d_counters != nullptr ? 2 : (pairs ? 1 : 0);
  // exact joins with cell-local refinement may resolve inside the probe;
  // the other refinement modes always use the resolve kernel
  const int pending = a->pending != ACT_PENDING_AUTO ? a->pending : L.pending;
  if (counts || ids) P.refine = ACT_REFINE_LOCAL;
  const int mode = counts ? (exact ? kExactCount : kApproxCount)
                   : ids ? (exact ? kExactList : kApprox)
                   : !exact ? kApprox
                   : (P.refine == ACT_REFINE_LOCAL && pending == ACT_PENDING_QUEUE) ? kExactFused
                                                                                    : kExactMask;
  int64_t pass = std::min(a->n, counts ? kCountPass : kMaxLaunchPoints);
  Workspace *w = nullptr;
  size_t lds_bytes = (size_t)n_lds * 1024;
  if (counts) {
    P.counts = counts;
    // the polygons' histogram joins the trie levels in LDS when it fits
    const int64_t hist = (int64_t)h.n_polys * 4;
    P.hist_bins = lds_bytes + hist <= (size_t)kLdsDynamicMax ? (int32_t)h.n_polys : 0;
    lds_bytes += (size_t)P.hist_bins * 4;
  }
  if (mode == kExactMask || mode == kExactCount || (ids && exact)) {
    if (ext) {
      w = ext;
    } else {
      rc = get_workspace(x, stream, std::max<int64_t>(a->n, kDefaultPass), false, w);
      if (rc) return rc;
    }
    P.mask = w->mask;
    P.plist = w->plist;
    P.pcount = w->pcount;
    pass = std::min(a->pass_points > 0 ? std::min(a->pass_points, w->cap) : w->cap,
                    counts || ids ? kCountPass : kMaxLaunchPoints);
  }
  if (ids) pass = std::min(pass, kCountPass);
  using ResolveFn = void (*)(ProbeParams, int64_t);
  const ResolveFn resolve = P.refine == ACT_REFINE_LOCAL
                              ? (count == 2   ? resolve_kernel<true, 2, false>
                                 : count == 1 ? resolve_kernel<true, 1, false>
                                              : resolve_kernel<true, 0, false>)
                              : (count == 2   ? resolve_kernel<false, 2, false>
                                 : count == 1 ? resolve_kernel<false, 1, false>
                                              : resolve_kernel<false, 0, false>);
  using ListFn = void (*)(ProbeParams, uint32_t);
  const ListFn resolve_list = count == 2   ? resolve_list_kernel<2>
                              : count == 1 ? resolve_list_kernel<1>
                                           : resolve_list_kernel<0>;
  for (int64_t s0 = 0; s0 < a->n; s0 += pass) {
    const int64_t n = std::min(pass, a->n - s0);
    P.pts = a->d_points ? (const double2 *)a->d_points + s0 : nullptr;
    P.ids = ids ? ids + s0 : nullptr;
    P.out = counts ? nullptr : a->d_out + s0;
    P.n = n;
    P.base = s0;
    const int64_t tile_blocks = (n + (int64_t)kProbeBlock * np - 1) / ((int64_t)kProbeBlock * np);
    int grid = (int)std::max<int64_t>(1, std::min<int64_t>(a->grid > 0 ? a->grid : L.grid,
                                                            tile_blocks));
    if (counts || ids) grid = std::min(grid, kCountGridMax);
    // cell-local refinement: the probe waves list their pending points when
    // the pass's indices fit 32 bits and the regions fit the workspace
    int pmode = mode;
    const int64_t nwaves = (int64_t)grid * kProbeWaves, tile_pts = 64 * (int64_t)np;
    const int64_t region = ((n + tile_pts - 1) / tile_pts + nwaves - 1) / nwaves * tile_pts;
    if (mode == kExactMask && P.refine == ACT_REFINE_LOCAL && n < (1ll << 32) &&
        nwaves <= kListWavesMax && region * nwaves <= w->plist_cap) {
      pmode = kExactList;
      P.region = (uint32_t)region;
    }
    if (mode == kExactCount || (ids && exact)) {
      if (!(n < (1ll << 32) && nwaves <= kListWavesMax && region * nwaves <= w->plist_cap))
        return fail(ACT_E_RANGE, "pending lists do not fit the workspace");
      P.region = (uint32_t)region;
    }
    const ProbeFn probe = counts ? probe_count_fn(exact, depth, np)
                          : ids  ? probe_ids_fn(exact, depth, np)
                                 : probe_fn(pmode, depth, count, np);
    hipLaunchKernelGGL(probe, dim3(grid), dim3(kProbeBlock), lds_bytes, (hipStream_t)stream, P);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess)
      return fail(ACT_E_HIP, std::string("probe launch: ") + hipGetErrorString(e));
    if (a->probe_event) HIP_TRY(hipEventRecord((hipEvent_t)a->probe_event, (hipStream_t)stream));
    if (pmode == kExactList || pmode == kExactCount) {
      const bool cnt = pmode == kExactCount;
      const ListFn list_fn = cnt ? resolve_list_kernel<0, true> : resolve_list;
      // a count join's resolve blocks each flush a histogram: fewer blocks
      const int64_t lgrid = std::min<int64_t>((nwaves + 3) / 4, cnt && P.hist_bins > 0 ? 1024 : 1ll << 30);
      hipLaunchKernelGGL(list_fn, dim3((unsigned)lgrid), dim3(kListBlock),
                         cnt ? (size_t)P.hist_bins * 4 : 0, (hipStream_t)stream, P,
                         (uint32_t)nwaves);
      e = hipGetLastError();
      if (e != hipSuccess)
        return fail(ACT_E_HIP, std::string("resolve launch: ") + hipGetErrorString(e));
      continue;
    }
    if (mode != kExactMask) continue;
    const int64_t nwords = (n + 63) / 64;
    const int64_t ranges = (nwords + kRangeWords - 1) / kRangeWords;
    hipLaunchKernelGGL(resolve, dim3((unsigned)std::min<int64_t>(ranges, 65535)),
                       dim3(kResolveBlock), 0, (hipStream_t)stream, P, nwords);
    e = hipGetLastError();
    if (e != hipSuccess)
      return fail(ACT_E_HIP, std::string("resolve launch: ") + hipGetErrorString(e));
  }
  return ACT_OK;
}

constexpr int kBatchGrid = 4096;  // fill / resolve blocks of a batched join

static int join_batched_impl(const act_index *x, const act_batch *d_batches, int32_t nb,
                             int64_t total_points, uint64_t *d_ticks, void *stream) {
  if (!x) return fail(ACT_E_ARG, "index is NULL");
  if (nb < 0 || total_points < 0) return fail(ACT_E_ARG, "nb < 0 or total_points < 0");
  if (nb > 0 && !d_batches) return fail(ACT_E_ARG, "batches is NULL");
  if (x->device < 0) return fail(ACT_E_DEVICE, "index was built without a device");
  int rc = check_stream_device(x, stream);
  if (rc) return rc;
  if (nb == 0) return ACT_OK;
  const HostIndex &h = x->host;
  const act_launch &L = x->launch;
  int depth = L.lds_levels < 0 ? default_lds_depth(h) : L.lds_levels;
  int n_lds = depth > 0 ? lds_nodes_for(h, depth) : 0;
  if (depth > 0 && n_lds <= 0) depth = n_lds = 0;
  DeviceGuard g(x->device);
  Workspace *w = nullptr;
  rc = get_batch_workspace(x, stream, nb, total_points, w);
  if (rc) return rc;
  const bool exact = h.mode == ACT_EXACT;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(batch_setup_kernel, dim3(1), dim3(kSetupBlock), 0, st, d_batches, nb,
                     w->cap_groups, w->vstart, w->vsorted, w->vorder, w->vhdr, d_ticks);
  hipLaunchKernelGGL(batch_fill_kernel, dim3(kBatchGrid), dim3(256), 0, st, w->vsorted, w->vorder,
                     nb, w->vhdr, w->group_batch);
  ProbeParams P{};
  index_params(x, ACT_REFINE_LOCAL, n_lds, P);  // batched: cell-local refinement
  P.batches = d_batches;
  P.group_batch = w->group_batch;
  P.vstart = w->vstart;
  P.vhdr = w->vhdr;
  P.gticks = d_ticks ? w->gticks : nullptr;
  const int mode = !exact ? kApprox : (L.pending == ACT_PENDING_QUEUE ? kExactFused : kExactMask);
  if (mode == kExactMask) P.mask = w->bmask;
  hipLaunchKernelGGL(probe_batched_fn(mode, depth, launch_np(x)), dim3(L.grid), dim3(kProbeBlock),
                     (size_t)n_lds * 1024, st, P);
  if (mode == kExactMask) {
    void (*resolve)(ProbeParams, int64_t) = resolve_kernel<true, 0, true>;
    hipLaunchKernelGGL(resolve, dim3(2048), dim3(kResolveBlock), 0, st, P, (int64_t)0);
  }
  if (d_ticks)
    hipLaunchKernelGGL(batch_finish_kernel, dim3((unsigned)std::min<int64_t>(((int64_t)nb + 3) / 4, 4096)),
                       dim3(256), 0, st, d_batches, w->vstart, nb, w->vhdr, w->gticks, d_ticks);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess)
    return fail(ACT_E_HIP, std::string("batched join launch: ") + hipGetErrorString(e));
  return ACT_OK;
}

// ------------------------------------------------------------- autotuner

// 64-bit digest of the index image (trie, lookup table, records, edges,
// mode): the key of the tuning cache.
static uint64_t index_digest(const HostIndex &h) {
  uint64_t d = 0x9e3779b97f4a7c15ull ^ (uint64_t)h.mode;
  auto mix = [&d](const void *p, size_t bytes) {
    const uint8_t *b = (const uint8_t *)p;
    size_t k = 0;
    for (; k + 8 <= bytes; k += 8) {
      uint64_t v;
      std::memcpy(&v, b + k, 8);
      d = (d ^ v) * 0x100000001b3ull;
      d ^= d >> 29;
    }
    for (; k < bytes; k++) d = (d ^ b[k]) * 0x100000001b3ull;
    d ^= (uint64_t)bytes * 0xff51afd7ed558ccdull;
  };
  mix(h.nodes.data(), h.nodes.size() * 8);
  mix(h.lut.data(), h.lut.size() * 4);
  mix(h.edges64.data(), h.edges64.size() * 8);
  mix(&h.precision_m, sizeof h.precision_m);
  mix(&h.geometry, sizeof h.geometry);
  return d;
}

static bool cache_lookup(const char *path, uint64_t key, act_launch &L) {
  if (!path) return false;
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  char arch[64];
  unsigned long long k;
  int g, lds, np, rf, pd;
  bool hit = false;
  while (std::fscanf(f, "%llx %63s %d %d %d %d %d", &k, arch, &g, &lds, &np, &rf, &pd) == 7)
    if (k == key && std::strcmp(arch, "gfx950") == 0 && g >= 1 && g <= 65536 && lds >= -1 &&
        lds <= 2 && (np == 1 || np == 2) && rf >= ACT_REFINE_LOCAL && rf <= ACT_REFINE_FP64 &&
        pd >= ACT_PENDING_KERNEL && pd <= ACT_PENDING_QUEUE) {  // other lines are skipped
      L.grid = g;
      L.lds_levels = lds;
      L.points_per_lane = np;
      L.refine = rf;
      L.pending = pd;
      hit = true;
    }
  std::fclose(f);
  return hit;
}

static void cache_store(const char *path, uint64_t key, const act_launch &L) {
  if (!path) return;
  FILE *f = std::fopen(path, "a");
  if (!f) return;
  std::fprintf(f, "%016llx gfx950 %d %d %d %d %d\n", (unsigned long long)key, L.grid,
               L.lds_levels, L.points_per_lane, L.refine, L.pending);
  std::fclose(f);
}

static int tune_impl(act_index *x, const double *d_sample, int64_t n, int32_t *d_out,
                     void *stream, const char *cache_path, act_tune_result *res) {
  if (!x || !res) return fail(ACT_E_ARG, "bad argument");
  if (n <= 0 || !d_sample || !d_out) return fail(ACT_E_ARG, "tuning needs a non-empty sample");
  if (x->device < 0) return fail(ACT_E_DEVICE, "index was built without a device");
  int rc = check_stream_device(x, stream);
  if (rc) return rc;
  std::memset(res, 0, sizeof *res);
  const uint64_t key = cache_path ? index_digest(x->host) : 0;
  act_launch best;
  if (cache_lookup(cache_path, key, best)) {
    x->launch = best;
    res->from_cache = 1;
  } else {
    DeviceGuard g(x->device);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    auto time_cfg = [&](const act_launch &L, float &ms) -> int {
      act_join_args a{};
      a.d_points = d_sample;
      a.n = n;
      a.d_out = d_out;
      a.refine = L.refine;
      a.grid = L.grid;
      a.lds_levels = L.lds_levels;
      a.points_per_lane = L.points_per_lane;
      a.pending = L.pending;
      int r = join_impl(x, &a, stream);  // warm
      if (r) return r;
      float t[3];
      for (int k = 0; k < 3; k++) {
        if (hipEventRecord(e0, st) != hipSuccess) return fail(ACT_E_HIP, "event record");
        r = join_impl(x, &a, stream);
        if (r) return r;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&t[k], e0, e1) != hipSuccess)
          return fail(ACT_E_HIP, "event timing");
      }
      std::sort(t, t + 3);
      ms = t[1];
      return ACT_OK;
    };
    const act_launch defaults;
    const act_launch saved = x->launch;
    x->launch = defaults;
    float ms;
    rc = time_cfg(defaults, ms);
    res->default_ms = ms;
    res->best_ms = ms;
    best = defaults;
    const int grids[] = {256, 512, 1024, 2048, 4096};
    const bool exact = x->host.mode == ACT_EXACT;
    for (int gi = 0; gi < 5 && !rc; gi++)
      for (int lds = 0; lds <= 2 && !rc; lds++) {
        if (lds > 0 && lds_nodes_for(x->host, lds) < 0) continue;
        for (int np = 1; np <= 2 && !rc; np++)
          for (int rf = ACT_REFINE_LOCAL; rf <= (exact ? ACT_REFINE_FP32_FILTER : ACT_REFINE_LOCAL) && !rc; rf++)
            for (int pd = ACT_PENDING_KERNEL;
                 pd <= (exact && rf == ACT_REFINE_LOCAL ? ACT_PENDING_QUEUE : ACT_PENDING_KERNEL) && !rc;
                 pd++) {
              act_launch L;
              L.grid = grids[gi];
              L.lds_levels = lds;
              L.points_per_lane = np;
              L.refine = rf;
              L.pending = pd;
              rc = time_cfg(L, ms);
              res->n_configs++;
              if (!rc && ms < res->best_ms) {
                res->best_ms = ms;
                best = L;
              }
            }
      }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) {
      x->launch = saved;
      return rc;
    }
    x->launch = best;
    cache_store(cache_path, key, best);
  }
  res->grid = best.grid;
  res->lds_levels = best.lds_levels;
  res->points_per_lane = best.points_per_lane;
  res->refine = best.refine;
  res->pending = best.pending;
  res->index_digest = key;
  return ACT_OK;
}

}  // namespace act

// ===================================================================== C ABI

using namespace act;

extern "C" {

void act_build_opts_init(act_build_opts *o) {
  if (!o) return;
  o->max_level = 20;
  o->device = 0;
  o->threads = 0;
  o->prefix_level = -1;
  o->margin_deg = 1e-9;
  o->train_points = nullptr;
  o->n_train = 0;
  o->memory_budget = 0;
  o->train_max_level = 30;
  o->geometry = ACT_GEOM_PLANE;
  o->max_covering_cells = 0;
  o->max_interior_cells = 256;
  o->max_interior_level = 20;
  o->reserved1 = 0;
}

// Builds the host index and, for a device, uploads it. ACT_AUTO follows the
// paper's policy (Section III-A): the approximate index at precision_m if
// its image fits opts->memory_budget, else the exact index trained within
// the budget, with the covering level lowered until the untrained image
// fits.
static int build_impl(const double *verts_latlng, const int64_t *ring_off,
                      const int32_t *poly_ring_off, int32_t n_polys, BuildParams bp,
                      act_index *x, std::string &err) {
  static const int32_t zero = 0;
  const int32_t *pro = n_polys > 0 ? poly_ring_off : &zero;
  int rc;
  try {
    if (bp.mode != ACT_AUTO) return build_host_index(verts_latlng, ring_off, pro, n_polys, bp, x->host, err);
    const int64_t budget = bp.memory_budget;
    BuildParams ap = bp;
    ap.mode = ACT_APPROX;
    ap.n_train = 0;
    // each cell of the covering takes at least one 8-byte trie entry
    ap.cell_limit = budget > 0 ? budget / 8 + 1 : 0;
    rc = build_host_index(verts_latlng, ring_off, pro, n_polys, ap, x->host, err);
    if (rc == ACT_OK && (budget == 0 || image_bytes(x->host) <= budget)) return ACT_OK;
    if (rc != ACT_OK && rc != ACT_E_RANGE) return rc;
    BuildParams ep = bp;
    ep.mode = ACT_EXACT;
    ep.precision_m = 0.0;
    for (int ml = bp.max_level; ml >= 1; ml -= 2) {
      ep.max_level = ml;
      rc = build_host_index(verts_latlng, ring_off, pro, n_polys, ep, x->host, err);
      if (rc) return rc;
      if (image_bytes(x->host) <= budget) return ACT_OK;
    }
    err = "no index fits the memory budget of " + std::to_string(budget) + " bytes";
    return ACT_E_RANGE;
  } catch (const std::bad_alloc &) {
    err = "out of host memory during build";
    return ACT_E_OOM;
  }
}

int act_build(const double *verts_latlng, const int64_t *ring_off, const int32_t *poly_ring_off,
              int32_t n_polys, int32_t mode, double precision_m, const act_build_opts *opts,
              act_index **out) {
  if (!out) return fail(ACT_E_ARG, "out is NULL");
  *out = nullptr;
  if (n_polys < 0) return fail(ACT_E_ARG, "n_polys < 0");
  if (n_polys > 0 && (!verts_latlng || !ring_off || !poly_ring_off))
    return fail(ACT_E_ARG, "polygon arrays are NULL");
  if (mode != ACT_EXACT && mode != ACT_APPROX && mode != ACT_AUTO)
    return fail(ACT_E_ARG, "mode must be ACT_EXACT, ACT_APPROX or ACT_AUTO");
  if (mode != ACT_EXACT && !(precision_m >= 0.05))
    return fail(ACT_E_ARG, "approximate mode needs precision_m >= 0.05");
  act_build_opts o;
  act_build_opts_init(&o);
  if (opts) o = *opts;
  BuildParams bp;
  bp.mode = mode;
  bp.precision_m = mode != ACT_EXACT ? precision_m : 0.0;
  bp.max_level = o.max_level ? o.max_level : 20;
  bp.threads = o.threads;
  bp.prefix_level = o.prefix_level;
  bp.margin_deg = o.margin_deg > 0 ? o.margin_deg : 1e-9;
  bp.train_points = o.train_points;
  bp.n_train = o.n_train;
  bp.memory_budget = o.memory_budget;
  bp.train_max_level = o.train_max_level ? o.train_max_level : 30;
  bp.geometry = o.geometry;
  bp.max_covering_cells = o.max_covering_cells;
  bp.max_interior_cells = o.max_interior_cells ? o.max_interior_cells : 256;
  bp.max_interior_level = o.max_interior_level ? o.max_interior_level : 20;
  if (bp.max_covering_cells < 0 || bp.max_interior_cells < 0 || bp.max_interior_level < 1 ||
      bp.max_interior_level > kMaxLevel)
    return fail(ACT_E_ARG, "covering budgets out of range");
  if (bp.max_covering_cells > 0 && mode != ACT_EXACT)
    return fail(ACT_E_ARG, "covering budgets apply to exact mode");
  if (bp.geometry != ACT_GEOM_PLANE && bp.geometry != ACT_GEOM_SPHERE)
    return fail(ACT_E_ARG, "geometry must be ACT_GEOM_PLANE or ACT_GEOM_SPHERE");
  if (bp.geometry == ACT_GEOM_SPHERE && mode != ACT_EXACT)
    return fail(ACT_E_ARG, "spherical geometry is supported in exact mode only");
  if (bp.n_train < 0 || (bp.n_train > 0 && !bp.train_points))
    return fail(ACT_E_ARG, "training needs n_train >= 0 points");
  if (bp.memory_budget < 0) return fail(ACT_E_ARG, "memory_budget < 0");
  if (mode == ACT_AUTO && bp.memory_budget <= 0)
    return fail(ACT_E_ARG, "ACT_AUTO needs a memory_budget");
  if (bp.train_max_level < 1 || bp.train_max_level > kMaxLevel)
    return fail(ACT_E_ARG, "train_max_level must be 1..30");
  const int device = o.device;
  if (bp.max_level < 1 || bp.max_level > kMaxLevel) return fail(ACT_E_ARG, "max_level must be 1..30");
  if (bp.prefix_level < -1 || bp.prefix_level > kMaxLevel)
    return fail(ACT_E_ARG, "prefix_level must be -1..30");
  if (!(bp.margin_deg > 0 && bp.margin_deg < 1e-3)) return fail(ACT_E_ARG, "margin_deg out of range");
  if (device >= 0 && device >= device_count())
    return fail(ACT_E_DEVICE, "HIP device " + std::to_string(device) + " not available");
  act_index *x = new (std::nothrow) act_index;
  if (!x) return fail(ACT_E_OOM, "out of host memory");
  std::string err;
  int rc = build_impl(verts_latlng, ring_off, poly_ring_off, n_polys, bp, x, err);
  if (rc) {
    delete x;
    return fail(rc, err);
  }
  x->device = device;
  if (device >= 0) {
    DeviceGuard g(device);
    rc = upload_image(x);
    if (rc) {
      free_image(x->dev);
      delete x;
      return rc;
    }
  }
  *out = x;
  return ACT_OK;
}

int act_save(const act_index *x, const char *path) {
  if (!x || !path) return fail(ACT_E_ARG, "index or path is NULL");
  std::string err;
  const int rc = save_host_index(x->host, &x->launch, sizeof(act_launch), path, err);
  return rc ? fail(rc, err) : ACT_OK;
}

int act_load(const char *path, int32_t device, act_index **out) {
  if (!path || !out) return fail(ACT_E_ARG, "path or out is NULL");
  *out = nullptr;
  if (device >= 0 && device >= device_count())
    return fail(ACT_E_DEVICE, "HIP device " + std::to_string(device) + " not available");
  act_index *x = new (std::nothrow) act_index;
  if (!x) return fail(ACT_E_OOM, "out of host memory");
  std::string err;
  act_launch L;
  int rc;
  try {
    rc = load_host_index(path, x->host, &L, sizeof L, err);
  } catch (const std::bad_alloc &) {
    rc = ACT_E_OOM;
    err = "out of host memory while loading";
  }
  if (rc) {
    delete x;
    return fail(rc, err);
  }
  const bool launch_ok = L.grid >= 1 && L.grid <= 65536 && L.lds_levels >= -1 &&
                         L.lds_levels <= 2 && (L.points_per_lane == 1 || L.points_per_lane == 2) &&
                         L.refine >= ACT_REFINE_LOCAL && L.refine <= ACT_REFINE_FP64 &&
                         L.pending >= ACT_PENDING_KERNEL && L.pending <= ACT_PENDING_QUEUE;
  x->launch = launch_ok ? L : act_launch();
  x->device = device;
  if (device >= 0) {
    DeviceGuard g(device);
    rc = upload_image(x);
    if (rc) {
      free_image(x->dev);
      delete x;
      return rc;
    }
  }
  *out = x;
  return ACT_OK;
}

void act_free(act_index *x) {
  if (!x) return;
  if (x->device >= 0) {
    DeviceGuard g(x->device);
    free_image(x->dev);
    for (auto &kv : x->ws) free_workspace(kv.second);
  }
  delete x;
}

int act_workspace_reserve(const act_index *x, void *stream, int64_t points) {
  if (!x) return fail(ACT_E_ARG, "index is NULL");
  if (points < 0 || points > (1ll << 40)) return fail(ACT_E_ARG, "points out of range");
  if (x->device < 0) return fail(ACT_E_DEVICE, "index was built without a device");
  int rc = check_stream_device(x, stream);
  if (rc) return rc;
  if (x->host.mode != ACT_EXACT) return ACT_OK;
  DeviceGuard g(x->device);
  Workspace *w = nullptr;
  return get_workspace(x, stream, std::max<int64_t>(points, 64), true, w);
}

int act_workspace_release(const act_index *x, void *stream) {
  if (!x) return fail(ACT_E_ARG, "index is NULL");
  if (x->device < 0) return fail(ACT_E_DEVICE, "index was built without a device");
  int rc = check_stream_device(x, stream);
  if (rc) return rc;
  DeviceGuard g(x->device);
  std::lock_guard<std::mutex> lk(x->ws_mu);
  auto it = x->ws.find(stream);
  if (it == x->ws.end()) return ACT_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing((hipStream_t)stream, &cs) == hipSuccess &&
      cs != hipStreamCaptureStatusNone)
    return fail(ACT_E_RANGE, "cannot release a workspace while its stream is being captured");
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  free_workspace(it->second);
  x->ws.erase(it);
  return ACT_OK;
}

int act_join_status(const int64_t *d_n_pairs, int64_t capacity, void *stream, int64_t *n_pairs) {
  if (!d_n_pairs || capacity < 0) return fail(ACT_E_ARG, "bad argument");
  int64_t m = 0;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(hipMemcpy(&m, d_n_pairs, sizeof m, hipMemcpyDeviceToHost));
  if (n_pairs) *n_pairs = m;
  if (m > capacity)
    return fail(ACT_E_OVERFLOW, std::to_string(m) + " pairs exceed the capacity of " +
                                    std::to_string(capacity));
  return ACT_OK;
}

int act_join_ex(const act_index *x, const act_join_args *args, void *stream) {
  return join_impl(x, args, stream);
}

int act_join_batched(const act_index *x, const act_batch *d_batches, int32_t nb,
                     int64_t total_points, uint64_t *d_ticks, void *stream) {
  return join_batched_impl(x, d_batches, nb, total_points, d_ticks, stream);
}

int act_tune(act_index *x, const double *d_sample, int64_t n, int32_t *d_out, void *stream,
             const char *cache_path, act_tune_result *result) {
  return tune_impl(x, d_sample, n, d_out, stream, cache_path, result);
}

int act_batched_reserve(const act_index *x, void *stream, int32_t max_batches,
                        int64_t max_points) {
  if (!x) return fail(ACT_E_ARG, "index is NULL");
  if (max_batches < 0 || max_points < 0) return fail(ACT_E_ARG, "negative size");
  if (x->device < 0) return fail(ACT_E_DEVICE, "index was built without a device");
  int rc = check_stream_device(x, stream);
  if (rc) return rc;
  DeviceGuard g(x->device);
  Workspace *w = nullptr;
  return get_batch_workspace(x, stream, std::max(max_batches, 1), max_points, w);
}

int act_batched_status(const act_index *x, void *stream, int32_t *ok) {
  if (!x || !ok) return fail(ACT_E_ARG, "bad argument");
  std::lock_guard<std::mutex> lk(x->ws_mu);
  auto it = x->ws.find(stream);
  if (it == x->ws.end() || !it->second.vhdr) return fail(ACT_E_ARG, "no batched join on this stream");
  DeviceGuard g(x->device);
  int64_t hdr[2];
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(hipMemcpy(hdr, it->second.vhdr, sizeof hdr, hipMemcpyDeviceToHost));
  *ok = hdr[1] == 0;
  return ACT_OK;
}

int act_wall_clock_hz(int32_t device, double *hz) {
  if (!hz) return fail(ACT_E_ARG, "hz is NULL");
  if (device < 0 || device >= device_count()) return fail(ACT_E_DEVICE, "no such HIP device");
  int khz = 0;
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device));
  *hz = 1e3 * khz;
  return ACT_OK;
}

int act_join(const act_index *x, const double *d_points, int64_t n, int32_t *d_out, void *stream) {
  act_join_args a{};
  a.d_points = d_points;
  a.n = n;
  a.d_out = d_out;
  a.lds_levels = -1;
  return join_impl(x, &a, stream);
}

int act_join_noalloc(const act_index *x, const double *d_points, int64_t n, int32_t *d_out,
                     void *stream) {
  if (!x) return fail(ACT_E_ARG, "index is NULL");
  if (n > kNoAllocMaxPoints)
    return fail(ACT_E_RANGE, "act_join_noalloc: " + std::to_string(n) +
                                 " points exceed its limit of " +
                                 std::to_string(kNoAllocMaxPoints) + " per call");
  if (x->device < 0) return fail(ACT_E_DEVICE, "index was built without a device");
  uint64_t *mask = nullptr;
  int rc = noalloc_scratch(x->device, mask);
  if (rc) return rc;
  Workspace w;
  w.mask = mask;
  w.cap = kNoAllocMaxPoints;
  act_join_args a{};
  a.d_points = d_points;
  a.n = n;
  a.d_out = d_out;
  a.lds_levels = -1;
  return join_impl(x, &a, stream, &w);
}

int act_join_ids(const act_index *x, const uint64_t *d_ids, const double *d_points, int64_t n,
                 int32_t *d_out, void *stream) {
  if (!x) return fail(ACT_E_ARG, "index is NULL");
  if (n > 0 && !d_ids) return fail(ACT_E_ARG, "ids is NULL");
  act_join_args a{};
  a.d_points = d_points;
  a.n = n;
  a.d_out = d_out;
  a.lds_levels = -1;
  return join_impl(x, &a, stream, nullptr, nullptr, d_ids);
}

int act_join_count(const act_index *x, const double *d_points, int64_t n, int64_t *d_counts,
                   void *stream) {
  if (!x) return fail(ACT_E_ARG, "index is NULL");
  if (!d_counts && x->host.n_polys > 0) return fail(ACT_E_ARG, "counts is NULL");
  act_join_args a{};
  a.d_points = d_points;
  a.n = n;
  a.lds_levels = -1;
  return join_impl(x, &a, stream, nullptr, (unsigned long long *)d_counts);
}

int act_join_pairs(const act_index *x, const double *d_points, int64_t n, int32_t *d_out,
                   int64_t *d_pair_point, int32_t *d_pair_poly, int64_t capacity,
                   int64_t *d_n_pairs, void *stream) {
  if (!d_pair_point || !d_pair_poly || !d_n_pairs) return fail(ACT_E_ARG, "pair arrays are NULL");
  act_join_args a{};
  a.d_points = d_points;
  a.n = n;
  a.d_out = d_out;
  a.d_pair_point = d_pair_point;
  a.d_pair_poly = d_pair_poly;
  a.pair_capacity = capacity;
  a.d_n_pairs = d_n_pairs;
  a.lds_levels = -1;
  return join_impl(x, &a, stream);
}

int act_cell_ids(const double *d_points, int64_t n, uint64_t *d_ids, void *stream) {
  if (n < 0) return fail(ACT_E_ARG, "n < 0");
  if (n > 0 && (!d_points || !d_ids)) return fail(ACT_E_ARG, "points/ids is NULL");
  if (n == 0) return ACT_OK;
  if (device_count() <= 0) return fail(ACT_E_DEVICE, "no HIP device");
  static std::mutex mu;
  static uint16_t *tabs[64] = {nullptr};  // per device: Hilbert table, then the trig table
  static double2 *trigs[64] = {nullptr};
  int dev = 0;
  if (stream) {
    if (hipStreamGetDevice((hipStream_t)stream, &dev) != hipSuccess) return fail(ACT_E_ARG, "invalid stream");
  } else {
    HIP_TRY(hipGetDevice(&dev));
  }
  if (dev < 0 || dev >= 64) return fail(ACT_E_DEVICE, "device index out of range");
  DeviceGuard g(dev);
  {
    std::lock_guard<std::mutex> lk(mu);
    if (!tabs[dev]) {
      uint16_t h[1024];
      hilbert_table4(h);
      std::vector<double2> t;
      trig_table(t);
      uint16_t *d = nullptr;
      double2 *dt = nullptr;
      HIP_TRY(hipMalloc((void **)&d, sizeof h));
      HIP_TRY(hipMemcpy(d, h, sizeof h, hipMemcpyHostToDevice));
      HIP_TRY(hipMalloc((void **)&dt, t.size() * sizeof(double2)));
      HIP_TRY(hipMemcpy(dt, t.data(), t.size() * sizeof(double2), hipMemcpyHostToDevice));
      trigs[dev] = dt;
      tabs[dev] = d;
    }
  }
  hipLaunchKernelGGL(cell_id_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream,
                     (const double2 *)d_points, n, tabs[dev], trigs[dev], d_ids);
  HIP_TRY(hipGetLastError());
  return ACT_OK;
}

int act_index_stats(const act_index *x, act_stats *o) {
  if (!x || !o) return fail(ACT_E_ARG, "NULL argument");
  const HostIndex &h = x->host;
  std::memset(o, 0, sizeof *o);
  o->n_polys = h.n_polys;
  o->n_edges = (int64_t)h.edges64.size() / 4;
  o->n_cells = h.n_cells;
  o->n_cells_interior_only = h.n_cells_interior_only;
  o->n_nodes = (int64_t)h.nodes.size() / 256;
  o->node_bytes = (int64_t)h.nodes.size() * 4;  // device entries are 32-bit
  o->lut_words = (int64_t)h.lut.size();
  o->edge_bytes = (int64_t)(h.edges32.size() * 4 + h.edges64.size() * 8);
  o->device_bytes = (int64_t)x->dev.bytes;
  o->max_depth = h.max_depth;
  o->max_refs = h.max_refs;
  o->max_cell_level = h.max_cell_level;
  for (int f = 0; f < 6; f++) {
    o->face_prefix_level[f] = h.faces[f].root >= 0 ? h.faces[f].plevel : -1;
    o->n_faces += h.faces[f].root >= 0;
  }
  o->mode = h.mode;
  const int depth = default_lds_depth(h);
  o->lds_nodes = depth > 0 ? lds_nodes_for(h, depth) : 0;
  o->precision_m = h.precision_m;
  o->build_seconds = h.build_seconds;
  o->local_words = h.local_words;
  o->train_splits = h.train_splits;
  o->train_points_used = h.train_points_used;
  o->image_bytes = image_bytes(h);
  o->margin_deg = h.margin_deg;
  o->geometry = h.geometry;
  return ACT_OK;
}

int act_lookup_host(const act_index *x, const int32_t *face, const uint32_t *i,
                    const uint32_t *j, int64_t n, uint64_t *entries) {
  if (!x || n < 0 || (n > 0 && (!face || !i || !j || !entries))) return fail(ACT_E_ARG, "bad argument");
  for (int64_t k = 0; k < n; k++) entries[k] = host_lookup(x->host, face[k], i[k], j[k]);
  return ACT_OK;
}

int act_refine_local_host(const act_index *x, int32_t face, uint32_t i, uint32_t j, double lat,
                          double lng, int32_t poly, int32_t *covered) {
  if (!x || !covered) return fail(ACT_E_ARG, "bad argument");
  const HostIndex &h = x->host;
  const uint64_t e = host_lookup(h, face, i, j);
  if ((e & kTagMask) != kTagLut || h.mode != ACT_EXACT)
    return fail(ACT_E_ARG, "no cell-local record for this cell");
  const uint32_t off = (uint32_t)(e >> 2);
  const uint32_t nt = h.lut[off], nc = h.lut[off + 1 + nt];
  for (uint32_t r = 0; r < nc; r++)
    if ((int32_t)h.lut[off + 2 + nt + r] == poly) {
      *covered = local_record_covers(&h.lut[h.lut[off + 2 + nt + nc + r]], lng, lat) ? 1 : 0;
      return ACT_OK;
    }
  return fail(ACT_E_ARG, "polygon is not a candidate of this cell");
}

int act_index_digest(const act_index *x, uint64_t *digest) {
  if (!x || !digest) return fail(ACT_E_ARG, "bad argument");
  *digest = index_digest(x->host);
  return ACT_OK;
}

int act_lut_host(const act_index *x, uint32_t *words, int64_t *n_words) {
  if (!x || !n_words) return fail(ACT_E_ARG, "bad argument");
  *n_words = (int64_t)x->host.lut.size();
  if (words) std::memcpy(words, x->host.lut.data(), x->host.lut.size() * 4);
  return ACT_OK;
}

int act_encode_refs_host(const uint32_t *refs, int32_t n_refs, uint32_t *lut, int64_t lut_cap,
                         int64_t *lut_len, uint64_t *entry) {
  if (!refs || n_refs <= 0 || !lut_len || !entry || *lut_len < 0 || *lut_len > lut_cap ||
      (lut_cap > 0 && !lut))
    return fail(ACT_E_ARG, "bad argument");
  std::vector<uint32_t> v(lut, lut + *lut_len);
  LutDedup *dd = lut_dedup_new();
  // rebuild the dedup map from the existing table (lists laid out back to back)
  std::vector<uint32_t> tmp;
  size_t off = 0;
  while (off < v.size()) {
    uint32_t nt = v[off];
    uint32_t nc = v[off + 1 + nt];
    std::vector<uint32_t> r;
    for (uint32_t k = 0; k < nt; k++) r.push_back((v[off + 1 + k] << 1) | 1u);
    for (uint32_t k = 0; k < nc; k++) r.push_back(v[off + 2 + nt + k] << 1);
    encode_refs(r.data(), (int)r.size(), tmp, dd);
    off += 2 + nt + nc;
  }
  uint64_t e = encode_refs(refs, n_refs, tmp, dd);
  lut_dedup_free(dd);
  if ((int64_t)tmp.size() > lut_cap) return fail(ACT_E_RANGE, "lut capacity exceeded");
  std::memcpy(lut, tmp.data(), tmp.size() * 4);
  *lut_len = (int64_t)tmp.size();
  *entry = e;
  return ACT_OK;
}

int act_orient_fp32_host(const double *a, const double *b, const double *p, const double *origin,
                         float m_poly) {
  float ax = (float)(a[0] - origin[0]), ay = (float)(a[1] - origin[1]);
  float bx = (float)(b[0] - origin[0]), by = (float)(b[1] - origin[1]);
  float qx = (float)(p[0] - origin[0]), qy = (float)(p[1] - origin[1]);
  float m = std::max(m_poly, std::max(std::fabs(qx), std::fabs(qy)));
  return orient_sign_fp32_filter(ax, ay, bx, by, qx, qy, tier1_eta(m));
}

int act_orient_exact_host(const double *a, const double *b, const double *p) {
  return orient_sign_exact(a[0], a[1], b[0], b[1], p[0], p[1]);
}

int act_orient_host_n(const double *abp, const double *origin, const float *m_poly, int64_t n,
                      int32_t tier, int8_t *out) {
  if (n < 0 || (n > 0 && (!abp || !out)) || tier < 0 || tier > 1 ||
      (tier == 1 && n > 0 && (!origin || !m_poly)))
    return fail(ACT_E_ARG, "bad argument");
  for (int64_t k = 0; k < n; k++) {
    const double *q = abp + 6 * k;
    out[k] = (int8_t)(tier == 0 ? orient_sign_exact(q[0], q[1], q[2], q[3], q[4], q[5])
                                : act_orient_fp32_host(q, q + 2, q + 4, origin + 2 * k, m_poly[k]));
  }
  return ACT_OK;
}

int act_abi_sizes(int64_t *sizes) {
  if (!sizes) return fail(ACT_E_ARG, "sizes is NULL");
  sizes[0] = (int64_t)sizeof(act_build_opts);
  sizes[1] = (int64_t)sizeof(act_join_args);
  sizes[2] = (int64_t)sizeof(act_stats);
  return ACT_OK;
}

const char *act_last_error(void) { return g_err.c_str(); }

const char *act_version(void) { return "act-mi355x 0.1 (gfx950)"; }

}  // extern "C"
