// probe.hip -- the GPU probe (Section III-E, Listings 2 and 3) for gfx950,
// and the C ABI around it.
//
// Per point (one lane each, grid-stride):
//   1. coalesced 16-byte load of (lat, lng) fp64;
//   2. domain check (non-finite / |lat| > 90 / |lng| > 180 -> no match);
//   3. fp64 projection lat/lng -> unit sphere -> cube face -> (u, v) ->
//      quadratic (s, t) -> 30-bit (i, j) (Section II, S2 paragraph);
//   4. Hilbert position via a 4-levels-per-step state table held in LDS;
//   5. stage 1 (Listing 4): face -> root, per-face common prefix check;
//   6. stage 2 (Listing 5): comparison-free descent, 8 key bits per node,
//      until a payload, a LUT offset or the sentinel;
//   7. stage 3: decode the tagged entry (Section III-E, three cases);
//   8. true hits (and every reference in approximate mode) are output;
//      candidate hits are refined by the crossing-number test of
//      Section II with the ST_Covers boundary rule: fp32 on
//      origin-translated coordinates with a proven error bound, fp64 +
//      exact arithmetic for the edges the bound leaves undecided;
//   9. out[i] = lowest matching id (or -1), further matches -> pair list.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
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
  uint64_t *nodes = nullptr;
  uint32_t *lut = nullptr;
  int32_t *eoff = nullptr;
  double2 *origin = nullptr;
  float *pm = nullptr;
  float4 *e32 = nullptr;
  double2 *e64 = nullptr;
  uint16_t *htab = nullptr;
  size_t bytes = 0;
};

}  // namespace act

struct act_index {
  act::HostIndex host;
  act::DevImage dev;
  int device = -1;
};

namespace act {

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
  const uint64_t *nodes;
  const uint32_t *lut;
  const int32_t *eoff;
  const double2 *origin;
  const float *pm;
  const float4 *e32;
  const double2 *e64;
  const uint16_t *htab;
  int32_t root[6];
  int32_t shift[6];  // 60 - 2 * prefix level
  uint64_t prefix[6];
  int32_t n_lds_nodes;  // trie nodes 1 .. n_lds_nodes staged in LDS
  int32_t refine;
};

constexpr int kBlock = 256;
constexpr int kWaves = kBlock / 64;

// --------------------------------------------------------- device math
//
// The projection needs fp64 (level-30 cells are 2^-30 of a face wide) but
// only to ~1e-13 relative: the builder's conservative cell boxes carry a
// 1e-9 degree margin. The pieces below are written for the argument ranges
// that occur and cost far fewer instructions than the general library
// routines.

// sin and cos of x degrees, |x| <= 180. Quadrant reduction in degrees is
// exact: r = x - 90 k with k = rint(x / 90) (Sterbenz: x and 90 k are within
// a factor of two when k != 0). Then t = r pi / 180, |t| <= pi/4 (+ rounding)
// and the Taylor series up to t^15 (sin) and t^16 (cos); truncation error
// below t^17/17! = 5e-17.
__device__ __forceinline__ void sincos_deg(double x, double &s, double &c) {
  const double k = rint(x * (1.0 / 90.0));
  const double r = fma(k, -90.0, x);
  const double t = r * 0.017453292519943295;  // pi / 180
  const double t2 = t * t;
  double ps = fma(t2, -1.0 / 1307674368000.0, 1.0 / 6227020800.0);  // -1/15!, 1/13!
  ps = fma(t2, ps, -1.0 / 39916800.0);                              // -1/11!
  ps = fma(t2, ps, 1.0 / 362880.0);                                 //  1/9!
  ps = fma(t2, ps, -1.0 / 5040.0);                                  // -1/7!
  ps = fma(t2, ps, 1.0 / 120.0);                                    //  1/5!
  ps = fma(t2, ps, -1.0 / 6.0);                                     // -1/3!
  const double sn = fma(t * t2, ps, t);
  double pc = fma(t2, 1.0 / 20922789888000.0, -1.0 / 87178291200.0);  // 1/16!, -1/14!
  pc = fma(t2, pc, 1.0 / 479001600.0);                                 //  1/12!
  pc = fma(t2, pc, -1.0 / 3628800.0);                                  // -1/10!
  pc = fma(t2, pc, 1.0 / 40320.0);                                     //  1/8!
  pc = fma(t2, pc, -1.0 / 720.0);                                      // -1/6!
  pc = fma(t2, pc, 1.0 / 24.0);                                        //  1/4!
  pc = fma(t2, pc, -0.5);
  const double cs = fma(t2, pc, 1.0);
  // rotate by q quarter turns: (sn, cs), (cs, -sn), (-sn, -cs), (-cs, sn)
  const int q = (int)k & 3;
  s = (q & 1) ? cs : sn;
  c = (q & 1) ? sn : cs;
  if (q & 2) s = -s;
  if ((q + 1) & 2) c = -c;
}

// 1 / a for a in [1/sqrt(3), 1]: hardware estimate + two Newton steps.
__device__ __forceinline__ double rcp_nr(double a) {
  double r = __builtin_amdgcn_rcp(a);
  double e = fma(-a, r, 1.0);
  r = fma(r, e, r);
  e = fma(-a, r, 1.0);
  return fma(r, e, r);
}

// sqrt(a) for a in [1, 4]: reciprocal square root estimate, two Newton
// steps on it, one multiply.
__device__ __forceinline__ double sqrt_nr(double a) {
  double y = __builtin_amdgcn_rsq(a);
  double h = fma(-a * y, y, 1.0);
  y = fma(0.5 * y, h, y);
  h = fma(-a * y, y, 1.0);
  y = fma(0.5 * y, h, y);
  return a * y;
}

// st(w) * 2^30 as a 30-bit cell coordinate.
__device__ __forceinline__ uint32_t leaf_coord(double w) {
  const double h = 0.5 * sqrt_nr(fma(3.0, fabs(w), 1.0));
  const double s = w >= 0.0 ? h : 1.0 - h;
  const uint32_t i = (uint32_t)fmax(s * kTwo30, 0.0);
  return min(i, (1u << 30) - 1u);
}

// Steps 2-4: leaf cell (face, 60-bit Hilbert key) of a point; false for
// points that are not finite or outside |lat| <= 90, |lng| <= 180.
__device__ __forceinline__ bool dev_leaf(double lat, double lng, const uint16_t *htab,
                                         uint32_t &face, uint64_t &key) {
  if (!(fabs(lat) <= 90.0 && fabs(lng) <= 180.0)) return false;
  double slat, clat, slng, clng;
  sincos_deg(lat, slat, clat);
  sincos_deg(lng, slng, clng);
  const double x = clat * clng, y = clat * slng, z = slat;
  const double ax = fabs(x), ay = fabs(y), az = fabs(z);
  const bool fx = ax >= ay && ax >= az;
  const bool fy = !fx && ay >= az;
  const double m = fx ? x : (fy ? y : z);
  const double c1 = fx ? y : (fy ? z : x);
  const double c2 = fx ? z : (fy ? x : y);
  face = (fx ? 0u : (fy ? 1u : 2u)) + (m < 0.0 ? 3u : 0u);
  const double r = rcp_nr(fabs(m));
  const uint32_t i = leaf_coord(c1 * r), j = leaf_coord(c2 * r);
  // Hilbert position, 4 levels per table step (32 padded levels: the two
  // leading zero levels leave the state unchanged and add zero digits).
  uint32_t e = 0, hi = 0, lo = 0;
#pragma unroll
  for (int sh = 28; sh >= 0; sh -= 4) {
    const uint32_t idx = (e & 0x300u) | (((i >> sh) & 15u) << 4) | ((j >> sh) & 15u);
    e = htab[idx];
    if (sh >= 16) hi = (hi << 8) | (e & 255u);
    else lo = (lo << 8) | (e & 255u);
  }
  key = ((uint64_t)hi << 32) | lo;
  return true;
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
template <bool COUNT>
__device__ __forceinline__ int edge_fp32_then_exact(const ProbeParams &P, int e, float qx, float qy,
                                                    float eta, double px, double py,
                                                    uint32_t &c_fp64, uint32_t &c_exact) {
  const float4 g = P.e32[e];  // ax ay bx by
  const bool a_up = g.y > qy, a_dn = g.y < qy;
  const bool b_up = g.w > qy, b_dn = g.w < qy;
  if ((a_up && b_up) || (a_dn && b_dn)) return 0;  // strictly above/below
  if ((a_up || a_dn) && (b_up || b_dn)) {           // strict straddle
    const int s = orient_sign_fp32_filter(g.x, g.y, g.z, g.w, qx, qy, eta);
    if (s != 0) return (b_up ? (s > 0) : (s < 0)) ? 1 : 0;
  }
  const double2 A = P.e64[2 * e], B = P.e64[2 * e + 1];
  if (COUNT) {
    c_fp64++;
    if (orient_sign_fp64_filter(A.x, A.y, B.x, B.y, px, py) == 0) c_exact++;
  }
  return edge_test_exact(A.x, A.y, B.x, B.y, px, py);
}

template <bool COUNT>
__device__ __forceinline__ int edge_fp64(const ProbeParams &P, int e, double px, double py,
                                         uint32_t &c_fp64, uint32_t &c_exact) {
  const double2 A = P.e64[2 * e], B = P.e64[2 * e + 1];
  if ((A.y > py && B.y > py) || (A.y < py && B.y < py)) return 0;
  if (COUNT) {
    c_fp64++;
    if (orient_sign_fp64_filter(A.x, A.y, B.x, B.y, px, py) == 0) c_exact++;
  }
  return edge_test_exact(A.x, A.y, B.x, B.y, px, py);
}

// Whole-wave point-in-polygon test of one (point, polygon) pair: lane l
// takes edges e0 + l, e0 + l + 64, ...; crossing parity = parity of the
// popcount of the toggle ballots; any lane on an edge decides "covered".
// Must be called by all 64 lanes with wave-uniform arguments.
template <bool COUNT>
__device__ bool wave_covers(const ProbeParams &P, int poly, double lat, double lng, int lane,
                            uint32_t &c_fp64, uint32_t &c_exact) {
  const int e0 = P.eoff[poly], e1 = P.eoff[poly + 1];
  const double px = lng, py = lat;
  uint32_t par = 0;
  if (P.refine == ACT_REFINE_FP32_FILTER) {
    const double2 o = P.origin[poly];
    const float qx = (float)(px - o.x), qy = (float)(py - o.y);
    const float eta = tier1_eta(fmaxf(P.pm[poly], fmaxf(fabsf(qx), fabsf(qy))));
    for (int base = e0; base < e1; base += 64) {
      const int e = base + lane;
      const int r = e < e1 ? edge_fp32_then_exact<COUNT>(P, e, qx, qy, eta, px, py, c_fp64, c_exact) : 0;
      if (ballot(r == 2)) return true;
      par ^= (uint32_t)__popcll(ballot(r == 1));
    }
  } else {
    for (int base = e0; base < e1; base += 64) {
      const int e = base + lane;
      const int r = e < e1 ? edge_fp64<COUNT>(P, e, px, py, c_fp64, c_exact) : 0;
      if (ballot(r == 2)) return true;
      par ^= (uint32_t)__popcll(ballot(r == 1));
    }
  }
  return (par & 1u) != 0;
}

// Lowest match goes to out[i]; every other match becomes a pair.
struct Hits {
  int32_t best = -1;
  __device__ __forceinline__ void add(const ProbeParams &P, int64_t i, int32_t poly) {
    if (best < 0) {
      best = poly;
      return;
    }
    const int32_t other = poly < best ? best : poly;
    best = poly < best ? poly : best;
    if (P.pair_pt) {
      const unsigned long long k = atomicAdd((unsigned long long *)P.n_pairs, 1ull);
      if ((int64_t)k < P.cap) {
        P.pair_pt[k] = i;
        P.pair_poly[k] = other;
      }
    }
  }
};

// Steps 5-6: face root, prefix check and descent. The first LDS_DEPTH node
// levels are read from the LDS copy of nodes 1 .. n_lds_nodes (breadth-first
// numbering puts the top levels first).
template <int LDS_DEPTH>
__device__ __forceinline__ uint64_t descend(const ProbeParams &P, const uint64_t *s_nodes,
                                            int root, int sh, uint64_t key, uint32_t &reads) {
  uint64_t node = (uint64_t)root, e = 0;
#pragma unroll
  for (int d = 0; d < LDS_DEPTH; d++) {
    sh -= 8;
    e = s_nodes[(node - 1) * 256 + ((key >> sh) & 255u)];
    reads++;
    if ((e & kTagMask) != kTagPtr || e == 0) return e;
    node = e >> 2;
  }
  for (;;) {
    sh -= 8;
    e = P.nodes[node * 256 + ((key >> sh) & 255u)];
    reads++;
    if ((e & kTagMask) != kTagPtr || e == 0) return e;
    node = e >> 2;
  }
}

// The probe. Each wavefront walks tiles of 64 consecutive points (one per
// lane), so every lane of a wave executes the same number of iterations and
// the cooperative refinement can use whole-wave ballots.
template <bool EXACT, int LDS_DEPTH, bool COUNT>
__global__ __launch_bounds__(kBlock) void probe_kernel(ProbeParams P) {
  extern __shared__ uint64_t s_nodes[];
  __shared__ uint16_t s_htab[1024];
  __shared__ uint64_t s_prefix[6];
  __shared__ int32_t s_root[6], s_shift[6];
  __shared__ int32_t q_poly[kWaves][64];
  __shared__ double q_lat[kWaves][64], q_lng[kWaves][64];
  for (int k = threadIdx.x; k < 1024; k += kBlock) s_htab[k] = P.htab[k];
  if (LDS_DEPTH > 0)
    for (int k = threadIdx.x; k < P.n_lds_nodes * 256; k += kBlock) s_nodes[k] = P.nodes[256 + k];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int f = 0; f < 6; f++) {
      s_prefix[f] = P.prefix[f];
      s_root[f] = P.root[f];
      s_shift[f] = P.shift[f];
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t c_pts = 0, c_inv = 0, c_false = 0, c_true = 0, c_candpts = 0, c_cand = 0,
           c_edges = 0, c_fp64 = 0, c_exact = 0, c_reads = 0, c_lut = 0;
  const int64_t ntiles = (P.n + 63) >> 6;
  const int64_t nwaves = (int64_t)gridDim.x * kWaves;
  for (int64_t tile = (int64_t)blockIdx.x * kWaves + wid; tile < ntiles; tile += nwaves) {
    const int64_t i = tile * 64 + lane;
    const bool live = i < P.n;
    double lat = 0.0, lng = 0.0;
    if (live) {
      const double2 pt = P.pts[i];
      lat = pt.x;
      lng = pt.y;
    }
    uint32_t face = 0;
    uint64_t key = 0, e = 0;
    const bool valid = live && dev_leaf(lat, lng, s_htab, face, key);
    if (valid) {
      const int sh = s_shift[face], root = s_root[face];
      if (root >= 0 && (key >> sh) == s_prefix[face])
        e = descend<LDS_DEPTH>(P, s_nodes, root, sh, key, c_reads);
    }
    if (COUNT) {
      c_pts += live;
      c_inv += live && !valid;
      c_false += valid && e == 0;
    }
    // stage 3: decode the entry; true hits (approx: all references) out
    Hits hits;
    const uint32_t tag = (uint32_t)(e & kTagMask);
    uint32_t cand0 = 0, cand1 = 0, lut_cand = 0;
    int ncand = 0;
    bool from_lut = false;
    if (e != 0 && tag != kTagLut) {
      const uint32_t r0 = (uint32_t)((e >> 2) & 0x7fffffffu);
      if (!EXACT || (r0 & 1u)) hits.add(P, i, (int32_t)(r0 >> 1));
      else cand0 = r0 >> 1, ncand = 1;
      if (tag == kTagTwo) {
        const uint32_t r1 = (uint32_t)((e >> 33) & 0x7fffffffu);
        if (!EXACT || (r1 & 1u)) hits.add(P, i, (int32_t)(r1 >> 1));
        else if (ncand == 0) cand0 = r1 >> 1, ncand = 1;
        else cand1 = r1 >> 1, ncand = 2;
      }
    } else if (tag == kTagLut) {
      const uint32_t off = (uint32_t)(e >> 2);
      const uint32_t nt = P.lut[off];
      for (uint32_t r = 0; r < nt; r++) hits.add(P, i, (int32_t)P.lut[off + 1 + r]);
      const uint32_t nc = P.lut[off + 1 + nt];
      if (!EXACT) {
        for (uint32_t r = 0; r < nc; r++) hits.add(P, i, (int32_t)P.lut[off + 2 + nt + r]);
      } else {
        ncand = (int)nc;
        lut_cand = off + 2 + nt;
        from_lut = true;
      }
      if (COUNT) c_lut++;
    }
    if (COUNT) {
      c_true += e != 0 && ncand == 0;
      c_candpts += ncand > 0;
      c_cand += ncand;
    }
    if (EXACT) {
      // candidates, one round per candidate rank: compact the wave's
      // candidates into its LDS queue, refine each with the whole wave
      for (int r = 0;; r++) {
        const bool has = r < ncand;
        const uint64_t mask = ballot(has);
        if (mask == 0) break;
        const int cnt = __popcll(mask);
        const int slot = lane_rank(mask);
        int32_t my_poly = 0;
        if (has) {
          my_poly = (int32_t)(from_lut ? P.lut[lut_cand + r] : (r == 0 ? cand0 : cand1));
          q_poly[wid][slot] = my_poly;
          q_lat[wid][slot] = lat;
          q_lng[wid][slot] = lng;
        }
        wave_sync();
        uint64_t covered = 0;
        for (int q = 0; q < cnt; q++) {
          const int poly = __builtin_amdgcn_readfirstlane(q_poly[wid][q]);
          if (COUNT && lane == 0) c_edges += (uint32_t)(P.eoff[poly + 1] - P.eoff[poly]);
          if (wave_covers<COUNT>(P, poly, q_lat[wid][q], q_lng[wid][q], lane, c_fp64, c_exact))
            covered |= 1ull << q;
        }
        wave_sync();
        if (has && ((covered >> slot) & 1ull)) hits.add(P, i, my_poly);
      }
    }
    if (live) P.out[i] = hits.best;
  }
  if (COUNT) {
    unsigned long long *C = P.counters;
    atomicAdd(C + ACT_CNT_POINTS, (unsigned long long)c_pts);
    atomicAdd(C + ACT_CNT_INVALID, (unsigned long long)c_inv);
    atomicAdd(C + ACT_CNT_FALSE_HIT, (unsigned long long)c_false);
    atomicAdd(C + ACT_CNT_SOLELY_TRUE, (unsigned long long)c_true);
    atomicAdd(C + ACT_CNT_CAND_POINTS, (unsigned long long)c_candpts);
    atomicAdd(C + ACT_CNT_CANDIDATES, (unsigned long long)c_cand);
    atomicAdd(C + ACT_CNT_EDGES, (unsigned long long)c_edges);
    atomicAdd(C + ACT_CNT_EDGE_FP64, (unsigned long long)c_fp64);
    atomicAdd(C + ACT_CNT_EDGE_EXACT, (unsigned long long)c_exact);
    atomicAdd(C + ACT_CNT_NODE_READS, (unsigned long long)c_reads);
    atomicAdd(C + ACT_CNT_LUT_READS, (unsigned long long)c_lut);
  }
}

__global__ __launch_bounds__(256) void cell_id_kernel(const double2 *pts, int64_t n,
                                                      const uint16_t *htab, uint64_t *ids) {
  __shared__ uint16_t s_htab[1024];
  for (int k = threadIdx.x; k < 1024; k += blockDim.x) s_htab[k] = htab[k];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
    double2 p = pts[i];
    uint32_t face;
    uint64_t key;
    ids[i] = dev_leaf(p.x, p.y, s_htab, face, key) ? (((uint64_t)face << 61) | (key << 1) | 1ull) : 0ull;
  }
}

using ProbeFn = void (*)(ProbeParams);
static ProbeFn probe_fn(bool exact, int lds_depth, bool count) {
  static const ProbeFn tab[2][3][2] = {
      {{probe_kernel<false, 0, false>, probe_kernel<false, 0, true>},
       {probe_kernel<false, 1, false>, probe_kernel<false, 1, true>},
       {probe_kernel<false, 2, false>, probe_kernel<false, 2, true>}},
      {{probe_kernel<true, 0, false>, probe_kernel<true, 0, true>},
       {probe_kernel<true, 1, false>, probe_kernel<true, 1, true>},
       {probe_kernel<true, 2, false>, probe_kernel<true, 2, true>}}};
  return tab[exact][lds_depth][count];
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
  void *ptrs[] = {d.nodes, d.lut, d.eoff, d.origin, d.pm, d.e32, d.e64, d.htab};
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

static int upload_image(act_index *x) {
  const HostIndex &h = x->host;
  DevImage &d = x->dev;
  uint16_t htab[1024];
  hilbert_table4(htab);
  int rc;
  if ((rc = upload(d.nodes, h.nodes.data(), h.nodes.size() * 8, d.bytes))) return rc;
  if ((rc = upload(d.lut, h.lut.data(), h.lut.size() * 4, d.bytes))) return rc;
  if ((rc = upload(d.eoff, h.poly_edge_off.data(), h.poly_edge_off.size() * 4, d.bytes))) return rc;
  if ((rc = upload(d.origin, h.poly_origin.data(), h.poly_origin.size() * 8, d.bytes))) return rc;
  if ((rc = upload(d.pm, h.poly_m.data(), h.poly_m.size() * 4, d.bytes))) return rc;
  if ((rc = upload(d.e32, h.edges32.data(), h.edges32.size() * 4, d.bytes))) return rc;
  if ((rc = upload(d.e64, h.edges64.data(), h.edges64.size() * 8, d.bytes))) return rc;
  if ((rc = upload(d.htab, htab, sizeof htab, d.bytes))) return rc;
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

constexpr int kLdsTrieBudget = 48 * 1024;

// Node count staged in LDS for `depth` levels (0 if it does not fit).
static int lds_nodes_for(const HostIndex &h, int depth) {
  int n = depth >= 2 ? h.n_d0 + h.n_d1 : (depth == 1 ? h.n_d0 : 0);
  return n * 2048 <= kLdsTrieBudget ? n : -1;
}

static int default_lds_depth(const HostIndex &h) {
  for (int d = 2; d >= 1; d--)
    if (lds_nodes_for(h, d) > 0) return d;
  return 0;
}

static int join_impl(const act_index *x, const act_join_args *a, void *stream) {
  if (!x) return fail(ACT_E_ARG, "index is NULL");
  if (!a) return fail(ACT_E_ARG, "args is NULL");
  if (a->n < 0) return fail(ACT_E_ARG, "n < 0");
  if (x->device < 0) return fail(ACT_E_DEVICE, "index was built without a device");
  if (a->n > 0 && (!a->d_points || !a->d_out)) return fail(ACT_E_ARG, "points/out is NULL");
  bool pairs = a->d_pair_point || a->d_pair_poly || a->d_n_pairs;
  if (pairs && (!a->d_pair_point || !a->d_pair_poly || !a->d_n_pairs || a->pair_capacity < 0))
    return fail(ACT_E_ARG, "pair output needs point, poly, counter arrays and capacity >= 0");
  if (a->refine != ACT_REFINE_FP32_FILTER && a->refine != ACT_REFINE_FP64)
    return fail(ACT_E_ARG, "unknown refine mode");
  if (a->block != 0 && a->block != kBlock) return fail(ACT_E_ARG, "block must be 0 or 256");
  if (a->grid < 0 || a->grid > 65536) return fail(ACT_E_ARG, "grid must be 0 .. 65536");
  const HostIndex &h = x->host;
  int depth = a->lds_levels < 0 ? default_lds_depth(h) : a->lds_levels;
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
  P.nodes = x->dev.nodes;
  P.lut = x->dev.lut;
  P.eoff = x->dev.eoff;
  P.origin = x->dev.origin;
  P.pm = x->dev.pm;
  P.e32 = x->dev.e32;
  P.e64 = x->dev.e64;
  P.htab = x->dev.htab;
  for (int f = 0; f < 6; f++) {
    const FaceRoot &F = h.faces[f];
    P.root[f] = F.root;
    P.shift[f] = 60 - 2 * F.plevel;
    P.prefix[f] = F.prefix;
  }
  P.n_lds_nodes = n_lds;
  P.refine = a->refine;
  int64_t tiles_blocks = (a->n + kBlock - 1) / kBlock;
  int grid = a->grid > 0 ? a->grid : 2048;
  grid = (int)std::max<int64_t>(1, std::min<int64_t>(grid, tiles_blocks));
  DeviceGuard g(x->device);
  ProbeFn fn = probe_fn(h.mode == ACT_EXACT, depth, a->d_counters != nullptr);
  hipLaunchKernelGGL(fn, dim3(grid), dim3(kBlock), (size_t)n_lds * 2048, (hipStream_t)stream, P);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(ACT_E_HIP, std::string("probe launch: ") + hipGetErrorString(e));
  return ACT_OK;
}

}  // namespace act

// ===================================================================== C ABI

using namespace act;

extern "C" {

int act_build(const double *verts_latlng, const int64_t *ring_off, const int32_t *poly_ring_off,
              int32_t n_polys, int32_t mode, double precision_m, const act_build_opts *opts,
              act_index **out) {
  if (!out) return fail(ACT_E_ARG, "out is NULL");
  *out = nullptr;
  if (n_polys < 0) return fail(ACT_E_ARG, "n_polys < 0");
  if (n_polys > 0 && (!verts_latlng || !ring_off || !poly_ring_off))
    return fail(ACT_E_ARG, "polygon arrays are NULL");
  if (mode != ACT_EXACT && mode != ACT_APPROX) return fail(ACT_E_ARG, "mode must be ACT_EXACT or ACT_APPROX");
  if (mode == ACT_APPROX && !(precision_m >= 0.05))
    return fail(ACT_E_ARG, "approximate mode needs precision_m >= 0.05");
  BuildParams bp;
  bp.mode = mode;
  bp.precision_m = mode == ACT_APPROX ? precision_m : 0.0;
  bp.max_level = 20;
  bp.threads = 0;
  bp.margin_deg = 1e-9;
  int device = 0;
  if (opts) {
    if (opts->max_level) bp.max_level = opts->max_level;
    bp.threads = opts->threads;
    if (opts->margin_deg > 0) bp.margin_deg = opts->margin_deg;
    device = opts->device;
  }
  if (bp.max_level < 1 || bp.max_level > kMaxLevel) return fail(ACT_E_ARG, "max_level must be 1..30");
  if (!(bp.margin_deg > 0 && bp.margin_deg < 1e-3)) return fail(ACT_E_ARG, "margin_deg out of range");
  if (device >= 0 && device >= device_count())
    return fail(ACT_E_DEVICE, "HIP device " + std::to_string(device) + " not available");
  act_index *x = new (std::nothrow) act_index;
  if (!x) return fail(ACT_E_OOM, "out of host memory");
  std::string err;
  static const int32_t zero = 0;
  int rc;
  try {
    rc = build_host_index(verts_latlng, ring_off, n_polys > 0 ? poly_ring_off : &zero, n_polys,
                          bp, x->host, err);
  } catch (const std::bad_alloc &) {
    rc = ACT_E_OOM;
    err = "out of host memory during build";
  }
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

void act_free(act_index *x) {
  if (!x) return;
  if (x->device >= 0) {
    DeviceGuard g(x->device);
    free_image(x->dev);
  }
  delete x;
}

int act_join_ex(const act_index *x, const act_join_args *args, void *stream) {
  return join_impl(x, args, stream);
}

int act_join(const act_index *x, const double *d_points, int64_t n, int32_t *d_out, void *stream) {
  act_join_args a{};
  a.d_points = d_points;
  a.n = n;
  a.d_out = d_out;
  a.lds_levels = -1;
  return join_impl(x, &a, stream);
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
  static uint16_t *tabs[64] = {nullptr};
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
      uint16_t *d = nullptr;
      HIP_TRY(hipMalloc((void **)&d, sizeof h));
      HIP_TRY(hipMemcpy(d, h, sizeof h, hipMemcpyHostToDevice));
      tabs[dev] = d;
    }
  }
  hipLaunchKernelGGL(cell_id_kernel, dim3(grid_for(n, 256)), dim3(256), 0, (hipStream_t)stream,
                     (const double2 *)d_points, n, tabs[dev], d_ids);
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
  o->node_bytes = (int64_t)h.nodes.size() * 8;
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
  o->precision_m = h.precision_m;
  o->build_seconds = h.build_seconds;
  return ACT_OK;
}

int act_lookup_host(const act_index *x, const uint64_t *ids, int64_t n, uint64_t *entries) {
  if (!x || n < 0 || (n > 0 && (!ids || !entries))) return fail(ACT_E_ARG, "bad argument");
  for (int64_t k = 0; k < n; k++) entries[k] = host_lookup(x->host, ids[k]);
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

const char *act_last_error(void) { return g_err.c_str(); }

const char *act_version(void) { return "act-mi355x 0.1 (gfx950)"; }

}  // extern "C"
