/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, brute-force CPU point/polygon join used to check the GPU
 * library. Only tests, the smoke check and the benchmark's CPU-baseline leg
 * load it; the product path never does. It shares no code with the library.
 *
 * What it computes (the plain definition the paper's join reaches exactly):
 *   for every point p and every polygon P, whether P covers p under the
 *   ST_Covers predicate (Section "Background": points on edges or vertices
 *   lie within the polygon). Geometry model: the plane x = longitude,
 *   y = latitude in degrees, straight edges, closed polygons; holes are
 *   rings of the same polygon and their edges are boundary too; inside-ness
 *   is the even-odd crossing number of the ray tracing test the paper names
 *   for refinement (Section "Background", PIP paragraph).
 *
 * All predicates are evaluated exactly on the given fp64 coordinates:
 *   orientation sign = sign of (bx-ax)(py-ay) - (by-ay)(px-ax), first with
 *   fp64 and the static error bound (3 + 16 eps) eps (|l| + |r|) from
 *   Shewchuk, "Adaptive Precision Floating-Point Arithmetic and Fast Robust
 *   Geometric Predicates" (1997), and when that bound does not decide, from
 *   an exact floating-point expansion of the determinant (error-free
 *   TwoSum / TwoProduct transformations, Knuth and Dekker; expansion growth
 *   per Shewchuk Theorem 10). Exact as long as no product underflows, i.e.
 *   nonzero coordinate differences above 2^-450.
 *
 * Points that are non-finite or outside |lat| <= 90, |lng| <= 180 match no
 * polygon.
 *
 * Built with gcc -O2 -fopenmp -ffp-contract=off (no FMA contraction: the
 * error-free transformations need exactly rounded products and sums).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_EPS 1.1102230246251565e-16 /* 2^-53, unit roundoff of fp64 */

/* ---- error-free transformations ---------------------------------------- */

/* s + e == a + b exactly (Knuth's TwoSum). */
static void or_two_sum(double a, double b, double *s, double *e) {
  double x = a + b;
  double bv = x - a;
  double av = x - bv;
  *e = (a - av) + (b - bv);
  *s = x;
}

/* p + e == a * b exactly (fused multiply-add gives the rounding error). */
static void or_two_prod(double a, double b, double *p, double *e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}

/* Add one double to a nonoverlapping expansion h[0..n) (increasing
 * magnitude); result is again nonoverlapping, length n + 1. */
static int or_grow(double *h, int n, double b) {
  double q = b;
  for (int i = 0; i < n; i++) {
    double s, e;
    or_two_sum(q, h[i], &s, &e);
    h[i] = e;
    q = s;
  }
  h[n] = q;
  return n + 1;
}

/* Exact sign of (bx-ax)(py-ay) - (by-ay)(px-ax). */
static int or_orient_exact(double ax, double ay, double bx, double by,
                           double px, double py) {
  double d[4][2];
  /* each difference as an exact pair hi + lo */
  or_two_sum(bx, -ax, &d[0][0], &d[0][1]);
  or_two_sum(py, -ay, &d[1][0], &d[1][1]);
  or_two_sum(by, -ay, &d[2][0], &d[2][1]);
  or_two_sum(px, -ax, &d[3][0], &d[3][1]);
  double h[40];
  int n = 0;
  for (int i = 0; i < 2; i++)
    for (int j = 0; j < 2; j++) {
      double p, e;
      or_two_prod(d[0][i], d[1][j], &p, &e);
      n = or_grow(h, n, e);
      n = or_grow(h, n, p);
      or_two_prod(d[2][i], d[3][j], &p, &e);
      n = or_grow(h, n, -e);
      n = or_grow(h, n, -p);
    }
  /* nonoverlapping expansion: the sign of the sum is the sign of its most
   * significant nonzero component */
  for (int i = n - 1; i >= 0; i--) {
    if (h[i] > 0) return 1;
    if (h[i] < 0) return -1;
  }
  return 0;
}

int oracle_orient_sign(double ax, double ay, double bx, double by, double px,
                       double py) {
  double l = (bx - ax) * (py - ay);
  double r = (by - ay) * (px - ax);
  double det = l - r;
  double bound = (3.0 + 16.0 * OR_EPS) * OR_EPS * (fabs(l) + fabs(r));
  if (det > bound) return 1;
  if (-det > bound) return -1;
  return or_orient_exact(ax, ay, bx, by, px, py);
}

/* Exact-only variant (no filter); used by tests to show the filter changes
 * nothing. */
int oracle_orient_sign_exact(double ax, double ay, double bx, double by,
                             double px, double py) {
  return or_orient_exact(ax, ay, bx, by, px, py);
}

/* Signs of n orientation tests (tests call this to check many cases at
 * once); abp holds (ax, ay, bx, by, px, py) for each test. */
void oracle_orient_sign_n(const double *abp, int64_t n, int exact_only, int8_t *out) {
  for (int64_t k = 0; k < n; k++) {
    const double *q = abp + 6 * k;
    out[k] = (int8_t)(exact_only ? or_orient_exact(q[0], q[1], q[2], q[3], q[4], q[5])
                                 : oracle_orient_sign(q[0], q[1], q[2], q[3], q[4], q[5]));
  }
}

/* ---- point in polygon ---------------------------------------------------- */

/* verts: interleaved (lat, lng). Returns 1 if polygon p covers (lat, lng).
 * use_bbox = 0 skips the bounding-box prefilter (a test shows it changes
 * nothing). */
static int or_covers(const double *verts, const int64_t *ring_off,
                     const int32_t *poly_ring_off, const double *bbox, int p,
                     double lat, double lng, int use_bbox) {
  if (use_bbox) {
    const double *b = bbox + 4 * (size_t)p; /* lat_min lat_max lng_min lng_max */
    if (lat < b[0] || lat > b[1] || lng < b[2] || lng > b[3]) return 0;
  }
  const double px = lng, py = lat;
  int inside = 0;
  for (int r = poly_ring_off[p]; r < poly_ring_off[p + 1]; r++) {
    int64_t k0 = ring_off[r], k1 = ring_off[r + 1];
    for (int64_t k = k0; k < k1; k++) {
      int64_t kn = (k + 1 < k1) ? k + 1 : k0; /* closing edge */
      double ay = verts[2 * k], ax = verts[2 * k + 1];
      double by = verts[2 * kn], bx = verts[2 * kn + 1];
      int straddle = (ay > py) != (by > py);
      int in_box = px >= fmin(ax, bx) && px <= fmax(ax, bx) &&
                   py >= fmin(ay, by) && py <= fmax(ay, by);
      if (!straddle && !in_box) continue;
      int s = oracle_orient_sign(ax, ay, bx, by, px, py);
      if (in_box && s == 0) return 1; /* on the boundary: covered */
      if (straddle && ((by > ay) ? (s > 0) : (s < 0))) inside ^= 1;
    }
  }
  return inside;
}

static int or_valid_point(double lat, double lng) {
  return isfinite(lat) && isfinite(lng) && fabs(lat) <= 90.0 &&
         fabs(lng) <= 180.0;
}

static double *or_bboxes(const double *verts, const int64_t *ring_off,
                         const int32_t *poly_ring_off, int n_polys) {
  double *bb = (double *)malloc(sizeof(double) * 4 * (size_t)(n_polys > 0 ? n_polys : 1));
  for (int p = 0; p < n_polys; p++) {
    double b[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (int r = poly_ring_off[p]; r < poly_ring_off[p + 1]; r++)
      for (int64_t k = ring_off[r]; k < ring_off[r + 1]; k++) {
        b[0] = fmin(b[0], verts[2 * k]);
        b[1] = fmax(b[1], verts[2 * k]);
        b[2] = fmin(b[2], verts[2 * k + 1]);
        b[3] = fmax(b[3], verts[2 * k + 1]);
      }
    memcpy(bb + 4 * (size_t)p, b, sizeof b);
  }
  return bb;
}

/* Covers test for a single (polygon, point); for tests. */
int oracle_covers(const double *verts, const int64_t *ring_off,
                  const int32_t *poly_ring_off, int32_t n_polys, int32_t p,
                  double lat, double lng, int use_bbox) {
  if (p < 0 || p >= n_polys || !or_valid_point(lat, lng)) return 0;
  double *bb = or_bboxes(verts, ring_off, poly_ring_off, n_polys);
  int c = or_covers(verts, ring_off, poly_ring_off, bb, p, lat, lng, use_bbox);
  free(bb);
  return c;
}

/*
 * The join. For each point i (interleaved lat, lng):
 *   out[i]   = lowest id of a covering polygon, or -1;
 *   cnt[i]   = number of covering polygons.
 * Pairs beyond out[i] are written, in (point, polygon) ascending order, to
 * pair_pt / pair_poly up to `capacity`; the total is returned in *n_pairs.
 * nthreads <= 0 uses the OpenMP default. Returns 0.
 */
int oracle_join(const double *verts, const int64_t *ring_off,
                const int32_t *poly_ring_off, int32_t n_polys,
                const double *pts, int64_t n, int32_t *out, int32_t *cnt,
                int64_t *pair_pt, int32_t *pair_poly, int64_t capacity,
                int64_t *n_pairs, int nthreads, int use_bbox) {
  double *bb = or_bboxes(verts, ring_off, poly_ring_off, n_polys);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; i++) {
    double lat = pts[2 * i], lng = pts[2 * i + 1];
    int32_t first = -1, c = 0;
    if (or_valid_point(lat, lng))
      for (int p = 0; p < n_polys; p++)
        if (or_covers(verts, ring_off, poly_ring_off, bb, p, lat, lng, use_bbox)) {
          if (first < 0) first = p;
          c++;
        }
    out[i] = first;
    cnt[i] = c;
  }
  /* second pass over the (rare) points with more than one covering polygon */
  int64_t m = 0;
  for (int64_t i = 0; i < n; i++) {
    if (cnt[i] < 2) continue;
    double lat = pts[2 * i], lng = pts[2 * i + 1];
    for (int p = out[i] + 1; p < n_polys; p++)
      if (or_covers(verts, ring_off, poly_ring_off, bb, p, lat, lng, use_bbox)) {
        if (m < capacity) {
          pair_pt[m] = i;
          pair_poly[m] = p;
        }
        m++;
      }
  }
  *n_pairs = m;
  free(bb);
  return 0;
}

/* ---- the spherical model ------------------------------------------------ */
/*
 * The paper refines candidates with S2's point-in-polygon test, which works
 * on the sphere (Section III-A). Reading of that model: a polygon's edges
 * are the minor great-circle arcs between consecutive vertices (unit
 * vectors of the vertices' lat/lng, by the C library's sin and cos); a
 * point lies within the polygon if it is a vertex, lies on an edge, or has
 * odd crossing parity along the arc from the point north on its meridian to
 * the pole (polygons contain no pole, so the pole is outside). The meridian
 * of the point meets edge (a, b) when the point's longitude is in the
 * edge's half-open longitude range [min, max) (edges along a meridian are
 * never crossed, only touched); it crosses the edge when the point and the
 * north pole lie on opposite sides of the edge's great circle, i.e. when
 * det(a, b, p) = p . (a x b) has the sign opposite to that of
 * det(a, b, N), which is the sign of lng_b - lng_a for edges shorter than
 * 180 degrees of longitude. det(a, b, p) = 0 with the point's longitude in
 * the closed range means the point is on the edge. det is evaluated in
 * fp64 on the computed unit vectors; points within rounding of an edge may
 * be decided either way (parity with the GPU is judged away from edges).
 */
static void or_unit(double lat, double lng, double v[3]) {
  const double d = 3.14159265358979323846 / 180.0;
  const double cp = cos(lat * d), sp = sin(lat * d), cl = cos(lng * d), sl = sin(lng * d);
  v[0] = cp * cl;
  v[1] = cp * sl;
  v[2] = sp;
}

static int or_covers_sphere(const double *verts, const int64_t *ring_off,
                            const int32_t *poly_ring_off, const double *bbox, int p,
                            double lat, double lng) {
  const double *bb = bbox + 4 * (size_t)p; /* arcs stay inside their longitude range */
  if (lng < bb[2] || lng > bb[3]) return 0;
  double q[3];
  or_unit(lat, lng, q);
  int inside = 0;
  for (int r = poly_ring_off[p]; r < poly_ring_off[p + 1]; r++) {
    int64_t k0 = ring_off[r], k1 = ring_off[r + 1];
    for (int64_t k = k0; k < k1; k++) {
      int64_t kn = (k + 1 < k1) ? k + 1 : k0;
      double alat = verts[2 * k], alng = verts[2 * k + 1];
      double blat = verts[2 * kn], blng = verts[2 * kn + 1];
      if ((lat == alat && lng == alng) || (lat == blat && lng == blng)) return 1; /* vertex */
      if (alng == blng) { /* along a meridian: touched, never crossed */
        if (lng == alng && lat >= fmin(alat, blat) && lat <= fmax(alat, blat)) return 1;
        continue;
      }
      double lo = fmin(alng, blng), hi = fmax(alng, blng);
      if (lng < lo || lng > hi) continue;
      double a[3], b[3];
      or_unit(alat, alng, a);
      or_unit(blat, blng, b);
      /* the great circle's normal as (b + a) x (b - a) = 2 (a x b): for
       * nearby endpoints b - a is exact (Sterbenz), so the normal keeps
       * full relative precision where a x b would cancel */
      const double s0 = b[0] + a[0], s1 = b[1] + a[1], s2 = b[2] + a[2];
      const double d0 = b[0] - a[0], d1 = b[1] - a[1], d2 = b[2] - a[2];
      const double n0 = s1 * d2 - s2 * d1;
      const double n1 = s2 * d0 - s0 * d2;
      const double n2 = s0 * d1 - s1 * d0;
      const double det = q[0] * n0 + q[1] * n1 + q[2] * n2;
      if (det == 0.0) return 1; /* on the edge's great circle, inside its range */
      if (lng == hi) continue;  /* half-open longitude range */
      const int s_pole = blng > alng ? 1 : -1;
      if ((det > 0 ? 1 : -1) == -s_pole) inside ^= 1;
    }
  }
  return inside;
}

int oracle_covers_sphere(const double *verts, const int64_t *ring_off,
                         const int32_t *poly_ring_off, int32_t n_polys, int32_t p,
                         double lat, double lng) {
  if (p < 0 || p >= n_polys || !or_valid_point(lat, lng)) return 0;
  double *bb = or_bboxes(verts, ring_off, poly_ring_off, n_polys);
  int c = or_covers_sphere(verts, ring_off, poly_ring_off, bb, p, lat, lng);
  free(bb);
  return c;
}

/* The join in the spherical model: outputs as oracle_join. */
int oracle_join_sphere(const double *verts, const int64_t *ring_off,
                       const int32_t *poly_ring_off, int32_t n_polys, const double *pts,
                       int64_t n, int32_t *out, int32_t *cnt, int64_t *pair_pt,
                       int32_t *pair_poly, int64_t capacity, int64_t *n_pairs, int nthreads) {
  double *bb = or_bboxes(verts, ring_off, poly_ring_off, n_polys);
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; i++) {
    double lat = pts[2 * i], lng = pts[2 * i + 1];
    int32_t first = -1, c = 0;
    if (or_valid_point(lat, lng))
      for (int p = 0; p < n_polys; p++)
        if (or_covers_sphere(verts, ring_off, poly_ring_off, bb, p, lat, lng)) {
          if (first < 0) first = p;
          c++;
        }
    out[i] = first;
    cnt[i] = c;
  }
  int64_t m = 0;
  for (int64_t i = 0; i < n; i++) {
    if (cnt[i] < 2) continue;
    double lat = pts[2 * i], lng = pts[2 * i + 1];
    for (int p = out[i] + 1; p < n_polys; p++)
      if (or_covers_sphere(verts, ring_off, poly_ring_off, bb, p, lat, lng)) {
        if (m < capacity) {
          pair_pt[m] = i;
          pair_poly[m] = p;
        }
        m++;
      }
  }
  *n_pairs = m;
  free(bb);
  return 0;
}

/* Great-circle distance in metres from (lat, lng) to the boundary (all
 * edges, as minor arcs) of polygon p: to the arc's great circle where the
 * point's foot lies between the endpoints, else to the nearer endpoint.
 * R = 6,371,008.8 m. For checking parity near edges. */
double oracle_boundary_dist_sphere_m(const double *verts, const int64_t *ring_off,
                                     const int32_t *poly_ring_off, int32_t p, double lat,
                                     double lng) {
  const double R = 6371008.8;
  double q[3];
  or_unit(lat, lng, q);
  double best = INFINITY;
  for (int r = poly_ring_off[p]; r < poly_ring_off[p + 1]; r++) {
    int64_t k0 = ring_off[r], k1 = ring_off[r + 1];
    for (int64_t k = k0; k < k1; k++) {
      int64_t kn = (k + 1 < k1) ? k + 1 : k0;
      double a[3], b[3];
      or_unit(verts[2 * k], verts[2 * k + 1], a);
      or_unit(verts[2 * kn], verts[2 * kn + 1], b);
      const double sa[3] = {b[0] + a[0], b[1] + a[1], b[2] + a[2]};
      const double da[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
      double n[3] = {sa[1] * da[2] - sa[2] * da[1], sa[2] * da[0] - sa[0] * da[2],
                     sa[0] * da[1] - sa[1] * da[0]};
      double nn = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
      double d;
      /* the foot of q on the great circle lies on the arc iff it is on the
       * inner side of both planes through n and an endpoint */
      double an[3] = {n[1] * a[2] - n[2] * a[1], n[2] * a[0] - n[0] * a[2], n[0] * a[1] - n[1] * a[0]};
      double nb[3] = {b[1] * n[2] - b[2] * n[1], b[2] * n[0] - b[0] * n[2], b[0] * n[1] - b[1] * n[0]};
      int on_arc = nn > 0 && (q[0] * an[0] + q[1] * an[1] + q[2] * an[2]) >= 0 &&
                   (q[0] * nb[0] + q[1] * nb[1] + q[2] * nb[2]) >= 0;
      if (on_arc) {
        double s = (q[0] * n[0] + q[1] * n[1] + q[2] * n[2]) / nn;
        d = fabs(asin(fmax(-1.0, fmin(1.0, s))));
      } else {
        double qa[3] = {q[1] * a[2] - q[2] * a[1], q[2] * a[0] - q[0] * a[2], q[0] * a[1] - q[1] * a[0]};
        double qb[3] = {q[1] * b[2] - q[2] * b[1], q[2] * b[0] - q[0] * b[2], q[0] * b[1] - q[1] * b[0]};
        double xa = atan2(sqrt(qa[0] * qa[0] + qa[1] * qa[1] + qa[2] * qa[2]),
                          q[0] * a[0] + q[1] * a[1] + q[2] * a[2]);
        double xb = atan2(sqrt(qb[0] * qb[0] + qb[1] * qb[1] + qb[2] * qb[2]),
                          q[0] * b[0] + q[1] * b[1] + q[2] * b[2]);
        d = fmin(xa, xb);
      }
      if (d * R < best) best = d * R;
    }
  }
  return best;
}

void oracle_boundary_dist_sphere_pairs(const double *verts, const int64_t *ring_off,
                                       const int32_t *poly_ring_off, const double *pts,
                                       const int64_t *pair_pt, const int32_t *pair_poly,
                                       int64_t m, double *dist) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < m; i++) {
    int64_t q = pair_pt[i];
    dist[i] = oracle_boundary_dist_sphere_m(verts, ring_off, poly_ring_off, pair_poly[i],
                                            pts[2 * q], pts[2 * q + 1]);
  }
}

/*
 * Checker for the approximate join: planar distance in metres from (lat, lng)
 * to the boundary (all ring edges) of polygon p, in the local equirectangular
 * frame at the point's latitude: X = dlng * cos(lat) * R * pi / 180,
 * Y = dlat * R * pi / 180, R = 6,371,008.8 m. The paper bounds the error of
 * the approximate join by the diagonal of the largest covering cell without
 * naming a metric; this is the reading used to check that bound.
 */
double oracle_boundary_dist_m(const double *verts, const int64_t *ring_off,
                              const int32_t *poly_ring_off, int32_t p,
                              double lat, double lng) {
  const double R = 6371008.8;
  const double k = R * 3.14159265358979323846 / 180.0;
  const double kx = k * cos(lat * 3.14159265358979323846 / 180.0);
  double best = INFINITY;
  for (int r = poly_ring_off[p]; r < poly_ring_off[p + 1]; r++) {
    int64_t k0 = ring_off[r], k1 = ring_off[r + 1];
    for (int64_t q = k0; q < k1; q++) {
      int64_t qn = (q + 1 < k1) ? q + 1 : k0;
      double ax = (verts[2 * q + 1] - lng) * kx, ay = (verts[2 * q] - lat) * k;
      double bx = (verts[2 * qn + 1] - lng) * kx, by = (verts[2 * qn] - lat) * k;
      double dx = bx - ax, dy = by - ay;
      double len2 = dx * dx + dy * dy;
      double t = len2 > 0 ? -(ax * dx + ay * dy) / len2 : 0.0;
      t = t < 0 ? 0 : (t > 1 ? 1 : t);
      double cx = ax + t * dx, cy = ay + t * dy;
      double d = sqrt(cx * cx + cy * cy);
      if (d < best) best = d;
    }
  }
  return best;
}

/* Batched form of the checker: dist[i] for pairs (pt[i], poly[i]). */
void oracle_boundary_dist_pairs(const double *verts, const int64_t *ring_off,
                                const int32_t *poly_ring_off, const double *pts,
                                const int64_t *pair_pt, const int32_t *pair_poly,
                                int64_t m, double *dist) {
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t i = 0; i < m; i++) {
    int64_t q = pair_pt[i];
    dist[i] = oracle_boundary_dist_m(verts, ring_off, poly_ring_off, pair_poly[i],
                                     pts[2 * q], pts[2 * q + 1]);
  }
}
