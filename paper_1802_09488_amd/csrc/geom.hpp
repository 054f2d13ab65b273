// geom.hpp -- orientation predicates and the point-in-polygon edge test used
// by the index builder (host) and the refinement tiers (GPU).
//
// Join predicate: ST_Covers (Section II) in the plane x = longitude,
// y = latitude (degrees), closed polygons, even-odd crossing number of a ray
// towards +x (the ray tracing PIP test, Section II). Per edge (a, b) and
// point p:
//   on boundary  <=> orient(a, b, p) == 0 and p inside the edge's closed box;
//   crossing     <=> (a.y > p.y) != (b.y > p.y) and p lies left of the
//                    upward-directed edge (orient > 0 for b.y > a.y,
//                    orient < 0 otherwise).
// orient(a, b, p) = (bx-ax)(py-ay) - (by-ay)(px-ax).
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>

#define ACT_HD __host__ __device__ __forceinline__

namespace act {

// ---------------------------------------------------------------------------
// Exact orientation sign in fp64 (builder, refinement tiers 2 and 3).
//
// Tier 2: fp64 evaluation with the static error bound (3 + 16 eps) eps
// (|l| + |r|), eps = 2^-53 (Shewchuk 1997, orient2d "ccwerrboundA").
// Tier 3: the determinant expanded into six products
//   bx*py - bx*ay - ax*py - by*px + by*ax + ay*px,
// each split exactly into value + rounding error with an FMA, the twelve
// terms summed without error into a nonoverlapping expansion; its most
// significant nonzero component carries the sign. Exact unless a product
// underflows (nonzero coordinates above 2^-450 in magnitude).
// ---------------------------------------------------------------------------

ACT_HD void exact_mul(double a, double b, double &p, double &e) {
  p = a * b;
  e = fma(a, b, -p);
}

ACT_HD void exact_add(double a, double b, double &s, double &e) {
#pragma clang fp contract(off)
  s = a + b;
  double z = s - a;
  e = (a - (s - z)) + (b - z);
}

// Grow a nonoverlapping expansion h[0..n) by b (exactly).
ACT_HD void expansion_grow(volatile double *h, int &n, double b) {
  double q = b;
  for (int i = 0; i < n; i++) {
    double s, e;
    exact_add(q, h[i], s, e);
    h[i] = e;
    q = s;
  }
  h[n++] = q;
}

// This path runs only when the fp64 filter cannot decide (exactly or nearly
// collinear inputs). The expansion lives in a small private array so that
// kernels carrying this code keep their register budget.
ACT_HD int orient_sign_expansion(double ax, double ay, double bx, double by,
                                 double px, double py) {
  volatile double h[12];
  int n = 0;
  const double f1[6] = {bx, -bx, -ax, -by, by, ay};
  const double f2[6] = {py, ay, py, px, ax, px};
  for (int k = 0; k < 6; k++) {
    double p, e;
    exact_mul(f1[k], f2[k], p, e);
    expansion_grow(h, n, e);
    expansion_grow(h, n, p);
  }
  for (int i = n - 1; i >= 0; i--) {
    const double v = h[i];
    if (v > 0.0) return 1;  // components ascend in magnitude
    if (v < 0.0) return -1;
  }
  return 0;
}

// Returns +1/-1 when the fp64 filter decides, 0 when it does not.
ACT_HD int orient_sign_fp64_filter(double ax, double ay, double bx, double by,
                                   double px, double py) {
#pragma clang fp contract(off)
  const double eps = 1.1102230246251565e-16;  // 2^-53
  double l = (bx - ax) * (py - ay);
  double r = (by - ay) * (px - ax);
  double det = l - r;
  double bound = (3.0 + 16.0 * eps) * eps * (fabs(l) + fabs(r));
  return det > bound ? 1 : (-det > bound ? -1 : 0);
}

ACT_HD int orient_sign_exact(double ax, double ay, double bx, double by,
                             double px, double py) {
  int s = orient_sign_fp64_filter(ax, ay, bx, by, px, py);
  return s != 0 ? s : orient_sign_expansion(ax, ay, bx, by, px, py);
}

// ---------------------------------------------------------------------------
// Tier 1: fp32 orientation on coordinates translated by a per-polygon fp64
// origin o and rounded to fp32 (the polygon's vertices once on the host, the
// point on the GPU: fp64 subtraction, then round-to-nearest to fp32).
//
// Error bound (derived for this code, contraction off, u = 2^-24):
//  * input rounding: |x_hat - (x - o)| <= eta with
//      eta = u (1 + 2^-20) M + 2^-100,
//    M >= every |x_hat| involved (fp64 then fp32 rounding of x - o; the
//    2^-100 term absorbs fp32 underflow);
//  * evaluation: d1 = bx-ax, d2 = py-ay, d3 = by-ay, d4 = px-ax (rounded),
//    t1 = d1 d2, t2 = d3 d4, det = t1 - t2 (rounded) differs from the exact
//    determinant D' of the rounded inputs by at most
//      (u + 3u/(1 - 6u)) (|t1| + |t2|) <= (4u + 32u^2)(|t1| + |t2|);
//  * input perturbation: each exact difference moves by <= 2 eta, so
//      |D' - D| <= 2 eta (|d1|+|d2|+|d3|+|d4|)/(1-u) + 8 eta^2,
//    D being the exact determinant of the original fp64 coordinates
//    (translation leaves it unchanged);
//  * the bound itself is evaluated in fp32: the result is inflated by
//    (1 + 16u) and an absolute 1e-30 covers product underflow.
// The sign of det is the exact sign whenever |det| > B.
// ---------------------------------------------------------------------------

ACT_HD float tier1_eta(float m) {
  return 5.9604644775390625e-08f * (1.0f + 9.5367431640625e-07f) * m +
         7.888609052210118e-31f;  // 2^-100
}

ACT_HD int orient_sign_fp32_filter(float ax, float ay, float bx, float by,
                                   float px, float py, float eta) {
#pragma clang fp contract(off)
  const float u = 5.9604644775390625e-08f;  // 2^-24
  float d1 = bx - ax, d2 = py - ay, d3 = by - ay, d4 = px - ax;
  float t1 = d1 * d2, t2 = d3 * d4;
  float det = t1 - t2;
  float s = fabsf(d1) + fabsf(d2) + fabsf(d3) + fabsf(d4);
  float B = (4.0f * u + 32.0f * u * u) * (fabsf(t1) + fabsf(t2)) +
            2.0f * eta * s * (1.0f + 2.0f * u) + 8.0f * eta * eta;
  B = B * (1.0f + 16.0f * u) + 1e-30f;
  return det > B ? 1 : (-det > B ? -1 : 0);
}

// ---------------------------------------------------------------------------
// One edge of the crossing-number test on original fp64 coordinates, with
// exact orientation (tiers 2 + 3). Returns 2 if p lies on the edge,
// 1 if the edge toggles the crossing parity, 0 otherwise.
// ---------------------------------------------------------------------------
ACT_HD int edge_test_exact(double ax, double ay, double bx, double by,
                           double px, double py) {
  bool straddle = (ay > py) != (by > py);
  bool in_box = px >= fmin(ax, bx) && px <= fmax(ax, bx) && py >= fmin(ay, by) &&
                py <= fmax(ay, by);
  if (!straddle && !in_box) return 0;
  int s = orient_sign_exact(ax, ay, bx, by, px, py);
  if (in_box && s == 0) return 2;
  if (straddle && ((by > ay) ? (s > 0) : (s < 0))) return 1;
  return 0;
}

// ---------------------------------------------------------------------------
// Cell-local refinement record (built by the index builder for a candidate
// (cell, polygon) pair): covered-ness of a point inside the cell's box from
// the edges that meet the box (exact tests), a base parity and the parity
// breakpoints of the edges passing right of the box. Record layout (32-bit
// words): n_local, n_break | base << 31, n_local x (ax ay bx by) fp64,
// n_break fp64 breakpoints.
// ---------------------------------------------------------------------------
ACT_HD double word_double(const uint32_t *w) {
  const uint64_t u = ((uint64_t)w[1] << 32) | w[0];
  double d;
  memcpy(&d, &u, sizeof d);
  return d;
}

ACT_HD bool local_record_covers(const uint32_t *rec, double px, double py) {
  const uint32_t n_local = rec[0], h1 = rec[1];
  const uint32_t n_break = h1 & 0x7fffffffu;
  uint32_t par = h1 >> 31;
  const uint32_t *d = rec + 2;
  for (uint32_t k = 0; k < n_local; k++, d += 8) {
    const int r = edge_test_exact(word_double(d), word_double(d + 2), word_double(d + 4),
                                  word_double(d + 6), px, py);
    if (r == 2) return true;
    par ^= (uint32_t)r;
  }
  for (uint32_t k = 0; k < n_break; k++, d += 2) par ^= word_double(d) <= py ? 1u : 0u;
  return par != 0;
}

// ---------------------------------------------------------------------------
// Closed segment vs closed axis-aligned box, exact (separating axes: the two
// box axes and the segment's normal).
// ---------------------------------------------------------------------------
ACT_HD bool segment_meets_box(double ax, double ay, double bx, double by,
                              double x0, double x1, double y0, double y1) {
  if (fmax(ax, bx) < x0 || fmin(ax, bx) > x1 || fmax(ay, by) < y0 ||
      fmin(ay, by) > y1)
    return false;
  int s0 = orient_sign_exact(ax, ay, bx, by, x0, y0);
  int s1 = orient_sign_exact(ax, ay, bx, by, x1, y0);
  int s2 = orient_sign_exact(ax, ay, bx, by, x1, y1);
  int s3 = orient_sign_exact(ax, ay, bx, by, x0, y1);
  if (s0 > 0 && s1 > 0 && s2 > 0 && s3 > 0) return false;
  if (s0 < 0 && s1 < 0 && s2 < 0 && s3 < 0) return false;
  return true;
}

}  // namespace act
