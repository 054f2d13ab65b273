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
  int32_t mode;
  int32_t refine;
};

// --------------------------------------------------------------- device

struct LdsTable {
  const uint16_t *t;
  __device__ uint16_t operator[](uint32_t k) const { return t[k]; }
};

// Steps 2-4: leaf cell of a point. Returns false for invalid points.
__device__ __forceinline__ bool dev_leaf(double lat, double lng, const uint16_t *htab,
                                         uint32_t &face, uint64_t &pos) {
  if (!(fabs(lat) <= 90.0 && fabs(lng) <= 180.0)) return false;
  double slat, clat, slng, clng;
  sincospi(lat * (1.0 / 180.0), &slat, &clat);
  sincospi(lng * (1.0 / 180.0), &slng, &clng);
  double x = clat * clng, y = clat * slng, z = slat;
  double ax = fabs(x), ay = fabs(y), az = fabs(z);
  double m, c1, c2;
  uint32_t a;
  if (ax >= ay && ax >= az) {
    a = 0; m = x; c1 = y; c2 = z;
  } else if (ay >= az) {
    a = 1; m = y; c1 = z; c2 = x;
  } else {
    a = 2; m = z; c1 = x; c2 = y;
  }
  face = a + (m < 0.0 ? 3u : 0u);
  double inv = 1.0 / fabs(m);
  double s = st_from_uv(c1 * inv), t = st_from_uv(c2 * inv);
  uint32_t i = (uint32_t)fmin(fmax(floor(s * kTwo30), 0.0), kTwo30 - 1.0);
  uint32_t j = (uint32_t)fmin(fmax(floor(t * kTwo30), 0.0), kTwo30 - 1.0);
  pos = hilbert_pos30(i, j, LdsTable{htab});
  return true;
}

// Point-in-polygon for a candidate (point, polygon) pair, ST_Covers rule.
// refine = ACT_REFINE_FP32_FILTER: fp32 tier first; undecided edges (equal
// rounded y / undecided orientation) are re-tested exactly in fp64.
__device__ bool dev_covers(const ProbeParams &P, int poly, double lat, double lng,
                           unsigned long long &c_edges, unsigned long long &c_fp64,
                           unsigned long long &c_exact) {
  const int e0 = P.eoff[poly], e1 = P.eoff[poly + 1];
  const double px = lng, py = lat;
  int inside = 0;
  c_edges += (unsigned long long)(e1 - e0);
  if (P.refine == ACT_REFINE_FP32_FILTER) {
    const double2 o = P.origin[poly];
    const float qx = (float)(px - o.x), qy = (float)(py - o.y);
    const float eta = tier1_eta(fmaxf(P.pm[poly], fmaxf(fabsf(qx), fabsf(qy))));
    for (int e = e0; e < e1; e++) {
      const float4 g = P.e32[e];  // ax ay bx by (translated)
      const bool a_up = g.y > qy, a_dn = g.y < qy;
      const bool b_up = g.w > qy, b_dn = g.w < qy;
      if ((a_up && b_up) || (a_dn && b_dn)) continue;  // edge entirely above/below
      int s = 0;
      if ((a_up || a_dn) && (b_up || b_dn)) s = orient_sign_fp32_filter(g.x, g.y, g.z, g.w, qx, qy, eta);
      if (s != 0) {
        // strict straddle and p off the edge's line: parity only
        if (b_up ? (s > 0) : (s < 0)) inside ^= 1;
        continue;
      }
      c_fp64++;
      const double2 A = P.e64[2 * e], B = P.e64[2 * e + 1];
      if (orient_sign_fp64_filter(A.x, A.y, B.x, B.y, px, py) == 0) c_exact++;
      int r = edge_test_exact(A.x, A.y, B.x, B.y, px, py);
      if (r == 2) return true;
      inside ^= r;
    }
  } else {
    for (int e = e0; e < e1; e++) {
      const double2 A = P.e64[2 * e], B = P.e64[2 * e + 1];
      if ((A.y > py && B.y > py) || (A.y < py && B.y < py)) continue;
      c_fp64++;
      if (orient_sign_fp64_filter(A.x, A.y, B.x, B.y, px, py) == 0) c_exact++;
      int r = edge_test_exact(A.x, A.y, B.x, B.y, px, py);
      if (r == 2) return true;
      inside ^= r;
    }
  }
  return inside != 0;
}

struct Hits {
  int32_t best = -1;
  __device__ void add(const ProbeParams &P, int64_t i, int32_t poly) {
    int32_t other;
    if (best < 0) {
      best = poly;
      return;
    }
    if (poly < best) {
      other = best;
      best = poly;
    } else {
      other = poly;
    }
    if (P.pair_pt) {
      unsigned long long k = atomicAdd((unsigned long long *)P.n_pairs, 1ull);
      if ((int64_t)k < P.cap) {
        P.pair_pt[k] = i;
        P.pair_poly[k] = other;
      }
    }
  }
};

__global__ __launch_bounds__(256) void probe_kernel(ProbeParams P) {
  __shared__ uint16_t s_htab[1024];
  __shared__ uint64_t s_prefix[6];
  __shared__ int32_t s_root[6], s_shift[6];
  for (int k = threadIdx.x; k < 1024; k += blockDim.x) s_htab[k] = P.htab[k];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int f = 0; f < 6; f++) {  // constant indices: read straight from kernel arguments
      s_prefix[f] = P.prefix[f];
      s_root[f] = P.root[f];
      s_shift[f] = P.shift[f];
    }
  }
  __syncthreads();
  unsigned long long c_inv = 0, c_false = 0, c_true = 0, c_candpts = 0, c_cand = 0, c_edges = 0,
                     c_fp64 = 0, c_exact = 0, c_nodes = 0, c_lut = 0, c_pts = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.n; i += stride) {
    const double2 pt = P.pts[i];
    const double lat = pt.x, lng = pt.y;
    c_pts++;
    uint32_t face;
    uint64_t key;
    Hits hits;
    if (!dev_leaf(lat, lng, s_htab, face, key)) {
      c_inv++;
      P.out[i] = -1;
      continue;
    }
    // stage 1: root and common prefix
    int sh = s_shift[face];
    int root = s_root[face];
    uint64_t e = 0;
    if (root >= 0 && (key >> sh) == s_prefix[face]) {
      // stage 2: descent
      uint64_t node = (uint64_t)root;
      for (;;) {
        sh -= 8;
        e = P.nodes[node * 256 + ((key >> sh) & 255u)];
        c_nodes++;
        if ((e & kTagMask) != kTagPtr || e == 0) break;
        node = e >> 2;
      }
    }
    if (e == 0) {
      c_false++;
      P.out[i] = -1;
      continue;
    }
    // stage 3: decode and emit
    const uint32_t tag = (uint32_t)(e & kTagMask);
    uint32_t inl[2];
    int n_inl = 0;
    bool any_cand = false;
    if (tag == kTagOne) {
      inl[0] = (uint32_t)((e >> 2) & 0x7fffffffu);
      n_inl = 1;
    } else if (tag == kTagTwo) {
      inl[0] = (uint32_t)((e >> 2) & 0x7fffffffu);
      inl[1] = (uint32_t)((e >> 33) & 0x7fffffffu);
      n_inl = 2;
    }
    for (int r = 0; r < n_inl; r++) {
      int32_t poly = (int32_t)(inl[r] >> 1);
      if ((inl[r] & 1u) || P.mode == ACT_APPROX) {
        hits.add(P, i, poly);
      } else {
        any_cand = true;
        c_cand++;
        if (dev_covers(P, poly, lat, lng, c_edges, c_fp64, c_exact)) hits.add(P, i, poly);
      }
    }
    if (tag == kTagLut) {
      c_lut++;
      uint32_t off = (uint32_t)(e >> 2);
      uint32_t nt = P.lut[off];
      for (uint32_t r = 0; r < nt; r++) hits.add(P, i, (int32_t)P.lut[off + 1 + r]);
      uint32_t nc = P.lut[off + 1 + nt];
      for (uint32_t r = 0; r < nc; r++) {
        int32_t poly = (int32_t)P.lut[off + 2 + nt + r];
        if (P.mode == ACT_APPROX) {
          hits.add(P, i, poly);
        } else {
          any_cand = true;
          c_cand++;
          if (dev_covers(P, poly, lat, lng, c_edges, c_fp64, c_exact)) hits.add(P, i, poly);
        }
      }
    }
    if (any_cand) c_candpts++;
    else c_true++;
    P.out[i] = hits.best;
  }
  if (P.counters) {
    unsigned long long *C = P.counters;
    atomicAdd(C + ACT_CNT_POINTS, c_pts);
    atomicAdd(C + ACT_CNT_INVALID, c_inv);
    atomicAdd(C + ACT_CNT_FALSE_HIT, c_false);
    atomicAdd(C + ACT_CNT_SOLELY_TRUE, c_true);
    atomicAdd(C + ACT_CNT_CAND_POINTS, c_candpts);
    atomicAdd(C + ACT_CNT_CANDIDATES, c_cand);
    atomicAdd(C + ACT_CNT_EDGES, c_edges);
    atomicAdd(C + ACT_CNT_EDGE_FP64, c_fp64);
    atomicAdd(C + ACT_CNT_EDGE_EXACT, c_exact);
    atomicAdd(C + ACT_CNT_NODE_READS, c_nodes);
    atomicAdd(C + ACT_CNT_LUT_READS, c_lut);
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
    uint64_t pos;
    ids[i] = dev_leaf(p.x, p.y, s_htab, face, pos) ? (((uint64_t)face << 61) | (pos << 1) | 1ull) : 0ull;
  }
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
  int block = a->block > 0 ? a->block : 256;
  if (block != 64 && block != 128 && block != 256)
    return fail(ACT_E_ARG, "block must be 64, 128 or 256");
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
    const FaceRoot &F = x->host.faces[f];
    P.root[f] = F.root;
    P.shift[f] = 60 - 2 * F.plevel;
    P.prefix[f] = F.prefix;
  }
  P.mode = x->host.mode;
  P.refine = a->refine;
  DeviceGuard g(x->device);
  hipLaunchKernelGGL(probe_kernel, dim3(grid_for(a->n, block)), dim3(block), 0,
                     (hipStream_t)stream, P);
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
