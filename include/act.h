/*
 * act.h -- C ABI of the MI355X Adaptive Cell Trie point/polygon join.
 *
 * Method: Kipf et al., "Adaptive Geospatial Joins for Modern Hardware"
 * (arXiv 1802.09488). The library builds, on the host, a precision-preserving
 * super covering of a set of polygons (Section III-B), stores it in an
 * Adaptive Cell Trie plus a lookup table (Section III-C), uploads that image
 * to HBM once, and probes streaming lat/lng points against it on the GPU
 * (Section III-E, Listings 2 and 3): point -> 64-bit cube-face/Hilbert cell
 * id -> trie descent -> true hits / candidate hits -> exact point-in-polygon
 * refinement of candidates. In approximate mode boundary cells are split
 * until their diagonal is below the requested precision and refinement is
 * skipped (Section III-A, approximate approach).
 *
 * Conventions shared by every entry point:
 *   - Coordinates are fp64 degrees, interleaved (lat, lng).
 *   - Join semantics are ST_Covers (Section II): a polygon covers the points
 *     on its edges and vertices, hole edges included; the plane is
 *     x = longitude, y = latitude with straight edges. Points that are not
 *     finite or lie outside |lat| <= 90, |lng| <= 180 match nothing.
 *   - Polygon ids are input positions 0 .. n_polys-1 (at most 2^30, the
 *     width of an inlined payload, Section III-C).
 *   - "Device pointer" means memory of the index's HIP device, owned by the
 *     caller; the library never frees it.
 *   - `stream` is a hipStream_t of the index's device (NULL = the default
 *     stream) passed as void*. Joins are enqueued asynchronously and never
 *     synchronise the host.
 *   - Every function returns ACT_OK (0) or a negative ACT_E_* code; the
 *     message of the last failure on the calling thread is returned by
 *     act_last_error(). Arguments are validated before anything is launched;
 *     on error nothing is launched and no output is written.
 *   - The index is immutable after act_build: concurrent joins on different
 *     streams or host threads are safe (Section IV-B1: probes of an
 *     immutable index need no synchronisation).
 */
#ifndef ACT_H
#define ACT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ACT_OK = 0,
  ACT_E_ARG = -1,      /* NULL pointer, n < 0, bad mode/precision/options   */
  ACT_E_POLY = -2,     /* malformed polygon input                            */
  ACT_E_OOM = -3,      /* host or device allocation failed                   */
  ACT_E_HIP = -4,      /* HIP runtime / launch error (message has details)   */
  ACT_E_OVERFLOW = -5, /* more result pairs than the caller's capacity       */
  ACT_E_DEVICE = -6,   /* no usable device, or index built without a device  */
  ACT_E_RANGE = -7     /* request beyond a documented limit                  */
};

/* ACT_AUTO: the paper's policy for a memory budget and a precision
 * (Section III-A): the approximate index at precision_m when its device
 * image fits act_build_opts.memory_budget, otherwise the exact index,
 * trained with the options' training points within the budget (Section
 * III-D); if even the untrained exact index does not fit, its covering
 * level is lowered (by two levels at a time) until it does. The built
 * index reports the mode it took (act_stats.mode). */
enum { ACT_EXACT = 0, ACT_APPROX = 1, ACT_AUTO = 2 };

/* Geometry of the polygons' edges. PLANE (default): straight segments in the
 * plane x = longitude, y = latitude (the ST_Covers reading, exact on the
 * input coordinates). SPHERE: minor great-circle arcs between the vertices,
 * as in S2's point-in-polygon test, which the paper uses for refinement
 * (Section III-A). A point is covered by a spherical polygon when it is a
 * vertex, lies on an edge, or when the arc from it north along its meridian
 * to the pole crosses the edges an odd number of times (polygons contain no
 * pole). Sign tests use fp64 unit vectors, so points within rounding of an
 * arc (about 1e-9 m) may be decided either way. Cells are classified
 * against the edges' chords with the cell margin widened by the largest
 * arc-to-chord distance, so true hits are true for the arcs too; candidates
 * are refined over all of the polygon's arcs (no cell-local records). */
enum { ACT_GEOM_PLANE = 0, ACT_GEOM_SPHERE = 1 };

/* Refinement of candidate hits in exact mode. All modes give identical,
 * exact results; they differ in cost. */
enum {
  ACT_REFINE_AUTO = 0,        /* ACT_REFINE_LOCAL                              */
  ACT_REFINE_LOCAL = 1,       /* cell-local test: only the polygon edges that
                                 meet the candidate cell's box are tested
                                 (exactly); the crossings of the remaining
                                 edges come from parity breakpoints the
                                 builder stored for the cell                  */
  ACT_REFINE_FP32_FILTER = 2, /* the crossing test over all of the polygon's
                                 edges (Section II ray tracing): fp32 with a
                                 proven error bound, fp64 re-test of undecided
                                 edges, exact expansion arithmetic last       */
  ACT_REFINE_FP64 = 3         /* all edges, every test in fp64 (+ exact)      */
};

typedef struct act_index act_index;

/* Build options; pass NULL for the defaults given per field. */
typedef struct {
  int32_t max_level;   /* exact mode: finest covering level (default 20;
                          Section V configuration uses 20 for interior
                          cells); range 1..30                                */
  int32_t device;      /* HIP device to upload to (default 0); -1 builds a
                          host-only index (inspection and tests; joins on it
                          return ACT_E_DEVICE)                               */
  int32_t threads;     /* host build threads (default 0 = hardware count)   */
  int32_t prefix_level; /* trie prefix level Lp of every face (Section III-D:
                          the face's cells share their first Lp levels,
                          nodes then cover levels Lp+1..Lp+4, Lp+5..Lp+8,
                          ...); -1 (default) = the common-ancestor level of
                          the face's cells, lowered (by at most 3) so that
                          the finest cells end a node level; an explicit
                          value is capped at the common-ancestor level      */
  double margin_deg;   /* conservative inflation of every cell's lat/lng box
                          before classification (default 1e-9 deg, which
                          covers fp64 projection rounding by >1e3x)          */
  /* Training (Section III-D), exact mode only: the index adapts to the
   * expected points. Each training point, in order, that falls into an
   * expensive cell (one with a candidate reference) splits that cell into
   * its four children, classified against the cell's references, until
   * the points run out or the next split would take the index's device
   * image beyond memory_budget. Ignored in approximate mode. */
  const double *train_points; /* host, 2 * n_train doubles (lat, lng); the
                                 array is read during act_build only       */
  int64_t n_train;            /* 0 (default): no training                  */
  int64_t memory_budget;      /* bytes of the device image (as
                                 act_stats.device_bytes); 0 = no limit.
                                 With ACT_AUTO also the approximate
                                 index's limit                             */
  int32_t train_max_level;    /* finest level training splits to (default
                                 30)                                       */
  int32_t geometry;           /* ACT_GEOM_PLANE (default) or ACT_GEOM_SPHERE
                                 (exact mode only)                         */
  /* Per-polygon coverings with cell budgets (exact mode), as the paper
   * configures them (Section V: 128 covering cells up to level 30, 256
   * interior cells up to level 20, with max_level = 30). 0 (default) builds
   * the joint subdivision instead, whose cells stop at max_level wherever a
   * polygon's boundary passes. Each polygon's covering is refined coarsest
   * cell first while its cell count stays within max_covering_cells (cells
   * inside the polygon are final); its interior covering keeps cells inside
   * the polygon, refined while within max_interior_cells and up to
   * max_interior_level; all coverings are merged without overlap, each cell
   * keeping the references of every covering cell it lies in (Section
   * III-B). Training (below) then refines the cells that the training
   * points find expensive. */
  int32_t max_covering_cells; /* 0 (default): no budget                   */
  int32_t max_interior_cells; /* default 256                               */
  int32_t max_interior_level; /* default 20                                */
  int32_t reserved1;
} act_build_opts;

/* Fills *opts with the defaults (the values act_build uses for NULL). */
void act_build_opts_init(act_build_opts *opts);

/*
 * act_build -- build an index over n_polys polygons (Sections III-B, III-C).
 *
 * verts_latlng  host, 2*V doubles: (lat, lng) of every vertex.
 * ring_off      host, R+1 int64: ring r spans vertices ring_off[r] ..
 *               ring_off[r+1]-1 (at least 3, closed implicitly).
 * poly_ring_off host, n_polys+1 int32: polygon p owns rings
 *               poly_ring_off[p] .. poly_ring_off[p+1]-1; the first is the
 *               outer ring, the rest are holes. Orientation is arbitrary.
 *               Polygons may overlap (a point then matches several).
 * mode          ACT_EXACT, ACT_APPROX or ACT_AUTO (needs a memory budget
 *               in opts).
 * precision_m   approx mode: every reported pair is a true containment or
 *               the point lies within precision_m metres of the polygon's
 *               boundary (cells are split until their diagonal is below
 *               it); must be >= 0.05. Ignored in exact mode.
 * out           receives the index; release it with act_free.
 *
 * Inputs are copied; the caller keeps ownership of its arrays. Polygons must
 * not cross the antimeridian or contain a pole (planar lat/lng model).
 * Consecutive duplicate vertices are dropped.
 * Errors: ACT_E_ARG, ACT_E_POLY (fewer than 3 distinct vertices in a ring,
 * non-finite or out-of-range coordinates, more than 2^30 polygons),
 * ACT_E_OOM, ACT_E_HIP, ACT_E_DEVICE, ACT_E_RANGE (ACT_AUTO: no index fits
 * the budget).
 */
int act_build(const double *verts_latlng, const int64_t *ring_off,
              const int32_t *poly_ring_off, int32_t n_polys, int32_t mode,
              double precision_m, const act_build_opts *opts,
              act_index **out);

/* Release an index and its device memory. NULL is a no-op. The caller must
 * make sure no join on it is still running. */
void act_free(act_index *idx);

/*
 * act_save / act_load -- an index as a file, so that a built (and trained,
 * and tuned) index can be reused without rebuilding. The file holds the
 * host image (trie, lookup table with the cell-local records, polygon
 * store, statistics) and the launch configuration act_tune chose, in a
 * little-endian binary layout with a version and a 64-bit digest.
 * act_load checks the digest and that every child pointer, list offset,
 * record and polygon id stays inside the image before uploading it to
 * `device` (-1: host only, as act_build_opts.device). The loaded index
 * equals the saved one (act_index_digest). Errors: ACT_E_ARG (NULL, cannot
 * open or write, not an index file, truncated or corrupt), ACT_E_OOM,
 * ACT_E_DEVICE, ACT_E_HIP.
 */
int act_save(const act_index *idx, const char *path);
int act_load(const char *path, int32_t device, act_index **out);

/*
 * act_join -- probe n points (Section III-E, Listing 3).
 *
 * d_points  device, 2*n doubles (lat, lng).
 * d_out     device, n int32: lowest id of a polygon that covers the point
 *           (exact mode) or that the point's cell references (approx mode),
 *           or -1.
 * n == 0 is a no-op. Further matches of a point (overlapping polygons,
 * shared edges and vertices) are not reported here; use act_join_pairs.
 * "Device" here means an address the kernels can use: device memory, or
 * pinned host memory at its device address (hipHostGetDevicePointer),
 * which the kernels then read and write over PCIe (the serving loop does
 * this for small groups). The results are in place once the stream has
 * passed the call.
 */
int act_join(const act_index *idx, const double *d_points, int64_t n,
             int32_t *d_out, void *stream);

/*
 * act_join_pairs -- as act_join, plus every match beyond d_out[i] as a
 * (point index, polygon id) pair (the paper's output is the list of join
 * pairs, Listing 3).
 *
 * d_pair_point, d_pair_poly  device arrays of `capacity` elements.
 * d_n_pairs  device int64 counter; the call adds the number of pairs it
 *            found (zero it first). Pairs beyond `capacity` are counted but
 *            not stored: after the stream completes, *d_n_pairs > capacity
 *            means the pair list is incomplete (ACT_E_OVERFLOW condition;
 *            rerun with a larger capacity). Pair order is unspecified.
 */
int act_join_pairs(const act_index *idx, const double *d_points, int64_t n,
                   int32_t *d_out, int64_t *d_pair_point, int32_t *d_pair_poly,
                   int64_t capacity, int64_t *d_n_pairs, void *stream);

/*
 * act_join_status -- the overflow check of a pair join: waits for `stream`,
 * reads the device pair counter `d_n_pairs` that act_join_pairs (or
 * act_join_ex with pair output) added to, and returns ACT_OK when every
 * pair was stored (counter <= capacity) or ACT_E_OVERFLOW when pairs were
 * dropped (rerun with a capacity of at least the counter). `n_pairs`
 * (optional, host) receives the counter. Errors: ACT_E_ARG, ACT_E_HIP.
 */
int act_join_status(const int64_t *d_n_pairs, int64_t capacity, void *stream,
                    int64_t *n_pairs);

/*
 * act_join_ids -- act_join for points that arrive with their level-30 cell
 * ids, as the points of the paper's probe do (Listing 3: each point carries
 * its cell id; the projection is not part of the probe there).
 *
 * d_ids     device, n uint64: the points' leaf cell ids in this library's
 *           layout (act_cell_ids): 3 face bits, the 60-bit Hilbert position,
 *           marker bit 1. An id that names no leaf (face above 5, bit 0
 *           clear, e.g. 0 for an invalid point) matches nothing.
 * d_points  device, 2*n doubles (lat, lng) of the same points: exact mode
 *           reads the points whose cells have candidates, to refine them;
 *           may be NULL in approximate mode.
 * d_out     device, n int32, as act_join.
 * The probe decodes each id to its leaf (face, i, j) and descends the trie
 * as act_join does; ids computed by any projection whose error stays within
 * the build's margin (act_build_opts.margin_deg) give act_join's results
 * (exact mode). Exact mode uses the stream's pending workspace. Errors as
 * act_join.
 */
int act_join_ids(const act_index *idx, const uint64_t *d_ids, const double *d_points,
                 int64_t n, int32_t *d_out, void *stream);

/*
 * act_join_count -- the paper's evaluation query, the number of points per
 * polygon (Section V: a count grouped by polygon id over the join pairs;
 * the aggregation follows the probe as in Section IV-B2, "produce output").
 *
 * d_points  device, 2*n doubles (lat, lng).
 * d_counts  device, n_polys int64 (NULL allowed only for an empty polygon
 *           set): the call ADDS to counts[p] the number of the points that
 *           polygon p covers (exact mode: every covering polygon of a point
 *           counts, overlaps and shared boundaries included, i.e. the pair
 *           set of act_join_pairs) or that reference p (approx mode: every
 *           reference of the point's cell). Zero it first for a plain
 *           count; repeated calls accumulate (streaming).
 * Writes no per-point output. Refinement is cell-local; in exact mode the
 * stream's pending workspace is used (allocated on first use, see
 * act_workspace_reserve). Counts are accumulated with atomics, so the
 * values are deterministic; the order of their updates is not. Errors as
 * act_join.
 */
int act_join_count(const act_index *idx, const double *d_points, int64_t n,
                   int64_t *d_counts, void *stream);

/*
 * act_join_noalloc -- act_join for callers that cannot allocate device
 * memory: code being captured into a HIP graph, tight serving loops,
 * harnesses that forbid hipMalloc. Same arguments and results as act_join;
 * it calls no hipMalloc, hipFree or other allocating routine, on any call.
 * Exact-mode joins keep their pending mask (one bit per point) in a static
 * device array of 16 MiB that the library holds on every device it runs on
 * until the process ends, instead of the stream's workspace, so:
 *   - n may be at most 2^27 (134,217,728) points per call; larger n returns
 *     ACT_E_RANGE before anything is launched;
 *   - all act_join_noalloc calls on one GPU share that array: calls that
 *     overlap in time on one GPU (different streams or host threads) race
 *     and must be serialised by the caller. Sequential calls need no
 *     clearing between them (each join writes every mask word it reads).
 * Pending points are always resolved by the mask's resolve kernel (or in
 * the probe's queues, when act_tune chose ACT_PENDING_QUEUE), never by the
 * per-wave lists. Errors as act_join, plus ACT_E_RANGE.
 */
int act_join_noalloc(const act_index *idx, const double *d_points, int64_t n,
                     int32_t *d_out, void *stream);

/*
 * act_workspace_reserve -- exact-mode joins record the points that need
 * refinement in a per-stream pending workspace owned by the index: a mask
 * (one bit per point of a pass) and per-wave pending lists (8 bytes per
 * point of a pass, plus 64 MiB). The first exact join on a stream allocates it for
 * max(n, 16 Mi) points; a later, longer join runs in passes of that many
 * points (no allocation). Call this beforehand to size it for `points`
 * points per pass, e.g. before capturing joins into a HIP graph, where
 * allocation is not allowed; enlarging an existing workspace synchronises
 * the stream first. No-op for approximate-mode indexes. Workspaces are
 * keyed by the stream handle and live until act_workspace_release or
 * act_free. Errors: ACT_E_ARG, ACT_E_DEVICE, ACT_E_OOM, ACT_E_HIP.
 */
int act_workspace_reserve(const act_index *idx, void *stream, int64_t points);

/*
 * act_workspace_release -- free the workspaces (pending mask and lists,
 * batched-join buffers) that joins on `stream` hold in this index, after
 * waiting for the work queued on the stream. Call it before destroying a
 * stream that ran joins: an index used from many short-lived streams
 * otherwise keeps one workspace per stream handle until act_free. A stream
 * without a workspace is a no-op; a later join on the stream allocates
 * again. Not allowed while the stream is being captured (ACT_E_RANGE).
 * Errors: ACT_E_ARG, ACT_E_DEVICE, ACT_E_RANGE, ACT_E_HIP.
 */
int act_workspace_release(const act_index *idx, void *stream);

/* Join counters (uint64 each), accumulated by act_join_ex when asked. */
enum {
  ACT_CNT_POINTS = 0,      /* points probed                                  */
  ACT_CNT_INVALID,         /* non-finite / out-of-range points               */
  ACT_CNT_FALSE_HIT,       /* trie returned no cell                          */
  ACT_CNT_SOLELY_TRUE,     /* cell with true hits only (no refinement)       */
  ACT_CNT_CAND_POINTS,     /* points with at least one candidate hit         */
  ACT_CNT_CANDIDATES,      /* candidate (point, polygon) pairs refined       */
  ACT_CNT_EDGES,           /* edges visited by refinement                    */
  ACT_CNT_EDGE_FP64,       /* edges the fp32 tier left undecided             */
  ACT_CNT_EDGE_EXACT,      /* edges the fp64 filter left undecided           */
  ACT_CNT_NODE_READS,      /* trie entries read (all levels, LDS included)   */
  ACT_CNT_LUT_READS,       /* cells whose references live in the LUT         */
  ACT_NCOUNTERS = 16
};

/* How an exact join resolves its pending points (points whose cell has
 * candidate references). KERNEL: the probe records them in the stream's
 * workspace (per-wave lists with cell-local refinement, else a mask) and a
 * second kernel refines them. QUEUE: each probe wave queues its
 * pending points in LDS and refines them itself, 64 at a time (no second
 * pass over the points; pays off when many points are pending). AUTO: the
 * index's launch configuration (KERNEL unless act_tune chose QUEUE). */
enum { ACT_PENDING_AUTO = 0, ACT_PENDING_KERNEL = 1, ACT_PENDING_QUEUE = 2 };

/* Full-control join; act_join / act_join_pairs are shorthands for it. */
typedef struct {
  const double *d_points;  /* device, 2*n doubles                            */
  int64_t n;
  int32_t *d_out;          /* device, n int32                                */
  int64_t *d_pair_point;   /* optional (NULL): pair output, see above        */
  int32_t *d_pair_poly;
  int64_t pair_capacity;
  int64_t *d_n_pairs;
  uint64_t *d_counters;    /* optional (NULL): ACT_NCOUNTERS accumulators    */
  int32_t refine;          /* ACT_REFINE_*                                   */
  int32_t block;           /* probe threads per block: 0 (default) or 1024  */
  int32_t lds_levels;      /* top trie node levels staged in LDS: 0, 1, 2, or
                              -1 for the default (deepest that fits 64 KiB
                              of 32-bit entries)                             */
  int32_t grid;            /* probe blocks launched (0 = default 1024); each
                              wave walks tiles of 64 points grid-stride      */
  int64_t pass_points;     /* exact joins with ACT_PENDING_KERNEL: points
                              per probe + resolve pass, at most the
                              workspace's (0 = the workspace's)              */
  int32_t points_per_lane; /* points each probe lane carries per step: 1, 2
                              (0 = default 2)                                */
  int32_t pending;         /* exact mode with cell-local refinement: how
                              pending points are resolved, ACT_PENDING_*
                              (other refinement modes always use the
                              kernel)                                        */
  void *probe_event;       /* optional hipEvent_t, recorded on the stream
                              after each probe launch (so, with
                              ACT_PENDING_KERNEL, between the probe and the
                              resolve kernel): lets a caller time the probe
                              alone                                          */
} act_join_args;

int act_join_ex(const act_index *idx, const act_join_args *args, void *stream);

/*
 * Batched joins (many point batches of uneven size in one pass over the
 * GPU, the streaming setting of Section V: the paper probes a large point
 * stream in parallel; here the stream arrives as batches).
 *
 * act_batch -- one batch: d_points (device, 2*n doubles, (lat, lng)
 * interleaved), n (>= 0), d_out (device, n int32: lowest covering polygon
 * id or -1, as act_join). Batches may not overlap in d_out.
 */
typedef struct {
  const double *d_points;
  int64_t n;
  int32_t *d_out;
} act_batch;

/*
 * act_join_batched -- join every batch of d_batches (a DEVICE array of nb
 * act_batch descriptors, caller-owned, read by the GPU during the call).
 * total_points must be at least the sum of the batches' n (it sizes the
 * workspace). One fixed set of launches on `stream` serves all batches
 * (setup, probe, resolve in exact mode, optional finish); the host reads
 * nothing back, so the call can be captured into a HIP graph once the
 * stream's workspace is large enough (act_batched_reserve) and replayed.
 * Batches are processed smallest first (by the bit length of their size;
 * input order within one length), so small batches complete early; the
 * results do not depend on the order.
 * d_ticks (optional, device, nb + 1 uint64): [0] the wall-clock tick at
 * which the join started on the GPU, [1 + b] the tick at which batch b was
 * complete (act_wall_clock_hz gives the tick rate). Extra matches of
 * overlapping polygons are not reported (out only). A call whose batch
 * sizes are negative or exceed the workspace writes nothing and leaves a
 * flag that act_batched_status reports. Errors: ACT_E_ARG, ACT_E_DEVICE,
 * ACT_E_OOM, ACT_E_RANGE (workspace too small while the stream is being
 * captured), ACT_E_HIP.
 */
int act_join_batched(const act_index *idx, const act_batch *d_batches, int32_t nb,
                     int64_t total_points, uint64_t *d_ticks, void *stream);

/* Size the stream's batched-join workspace for up to max_batches batches of
 * max_points points in total (synchronises the stream if it grows). */
int act_batched_reserve(const act_index *idx, void *stream, int32_t max_batches,
                        int64_t max_points);

/* Whether the stream's last batched join was well-formed (*ok = 1) or was
 * refused on the GPU (*ok = 0). Synchronises the stream. */
int act_batched_status(const act_index *idx, void *stream, int32_t *ok);

/*
 * act_tune -- autotuner. Times joins of the sample (device, 2*n doubles;
 * d_out: device scratch of n int32) over probe grid sizes (256 .. 4096
 * blocks), LDS-staged trie depth (0 .. 2, where the levels fit), points
 * per lane (1, 2) and, in exact mode, the refinement mapping (cell-local,
 * with pending points resolved by a second kernel or by the probe's own
 * queues, or all edges with the fp32 filter), picks the fastest (median of
 * 3) and makes it the index's launch configuration: joins that leave grid =
 * 0, lds_levels = -1, points_per_lane = 0, refine = ACT_REFINE_AUTO or
 * pending = ACT_PENDING_AUTO, and batched joins, use it from then on. The hand-tuning the paper reports for
 * its CPUs (Section V) is done by measurement here. With cache_path (a
 * text file, one line per (index digest, gfx950) -> configuration) a
 * cached configuration is applied without timing, and new results are
 * appended. Synchronises the stream. Do not tune an index while joins on
 * it are in flight. Errors: ACT_E_ARG, ACT_E_DEVICE, ACT_E_HIP.
 */
/* 64-bit digest of the index image (trie, lookup table, cell-local records,
 * edges, mode, precision): equal for equal inputs and build options, on any
 * thread count. */
int act_index_digest(const act_index *idx, uint64_t *digest);

typedef struct {
  int32_t grid, lds_levels, points_per_lane, refine;  /* chosen configuration */
  float best_ms;          /* its median join time on the sample              */
  float default_ms;       /* the built-in defaults' median join time         */
  int32_t n_configs;      /* configurations timed (0 when from the cache)    */
  int32_t from_cache;     /* 1 if read from cache_path                       */
  int32_t pending;        /* chosen ACT_PENDING_* (exact mode)               */
  int32_t reserved;
  uint64_t index_digest;  /* cache key (0 without cache_path)                */
} act_tune_result;

int act_tune(act_index *idx, const double *d_sample, int64_t n, int32_t *d_out, void *stream,
             const char *cache_path, act_tune_result *result);

/*
 * Serving loop (server.cpp): point-join requests of uneven size against
 * several resident indexes, admitted continuously and overlapping on the
 * GPU. A scheduler thread admits requests in arrival order when one of
 * `slots` streams is free and the request's buffers (20 bytes per point)
 * fit a device arena and a pinned host arena of `arena_bytes` each
 * (allocated once; 0 = 90% of free HBM, at most 4 GiB). When a slot frees
 * up, the request at the front of the queue is admitted together with the
 * requests for the same index waiting behind it (continuous batching: up to
 * max_request_points points in all, or the front request alone if it is
 * longer; up to 1024 requests). The group is staged into pinned memory;
 * a group of up to 2^16 points is joined (one act_join) straight from it,
 * the kernels reading the points and writing the results over PCIe, and a
 * larger one is copied to the GPU, joined and copied back, on the slot's
 * stream; each request's results land in its caller's h_out. A request's
 * result does not depend on the group it ran in.
 * Exact-mode workspaces for every (index, stream) are reserved at creation
 * for max_request_points (longer requests run in passes), so serving
 * allocates nothing, and the slots are warmed up (per slot, twice, all
 * slots in flight together: a join of min(max_request_points, 2^20,
 * arena / (20 * slots)) points at (0, 0) with each index on its stream,
 * with its copies), so the first requests do not pay the runtime's first
 * use of a stream. The pinned arena is written once at creation (its
 * pages are faulted in then, not during staging). The indexes must outlive
 * the server.
 */
typedef struct act_server act_server;

typedef struct {
  int32_t slots;               /* concurrent requests on the GPU (default 4)  */
  int32_t device;              /* HIP device (default 0)                      */
  int64_t arena_bytes;         /* per-arena bytes (default 0, see above)      */
  int64_t max_request_points;  /* workspace sizing and launch-group points
                                  (default 2^20)                              */
} act_server_opts;

/* A request's times (act_server_clock() seconds): arrival; admission (its
 * launch group took a slot and arena memory); launched (the group's points
 * staged and its copies and join enqueued); results (the group's results
 * found in pinned host memory); done (the request's results copied to its
 * h_out). */
typedef struct {
  double arrival_s, admitted_s, launched_s, results_s, done_s;
  int64_t n;
} act_request_times;

typedef struct {
  int64_t submitted, admitted, completed, failed, queued, points, arena_bytes;
  int32_t slots, reserved;
  int64_t launches;  /* launch groups (joins) started                        */
  /* the scheduler thread's longest pass through its loop (idle waits
   * excluded), and the longest it spent on one group's launch (staging
   * and enqueuing its copies and join), on the staging copies alone, and
   * on one group's completion (result copies), in seconds              */
  double max_pass_s, max_launch_s, max_stage_s, max_finish_s;
} act_server_stats;

void act_server_opts_init(act_server_opts *opts);
int act_server_create(const act_index *const *indexes, int32_t n_indexes,
                      const act_server_opts *opts, act_server **out);
/* Queue a request: n points at h_points (host, 2*n doubles) joined with
 * indexes[index]; results to h_out (host, n int32). Both buffers must stay
 * valid until act_server_wait returns for the ticket. arrival_s (seconds on
 * act_server_clock(), 0 = now) is the request's arrival time for latency.
 * ACT_E_RANGE if the request can never fit the arena (20 bytes a point,
 * rounded up to the arena's 256-byte granules). */
int act_server_submit(act_server *s, int32_t index, const double *h_points, int64_t n,
                      int32_t *h_out, double arrival_s, uint64_t *ticket);
/* Block until the request is complete; its times go to *t (may be NULL).
 * Each ticket is waited for exactly once. */
int act_server_wait(act_server *s, uint64_t ticket, act_request_times *t);
/*
 * act_server_replay -- a native load generator (measurements). Submits n
 * requests, request k at arrival_s[k] (act_server_clock seconds; the
 * calling thread spins until it is due, so the pacing does not depend on
 * the caller's runtime), joining n_points[k] points at h_points[k] (host,
 * 2*n_points[k] doubles) with indexes[index[k]]. A second thread waits for
 * the requests in order and writes each one's times to times[k] (host, n
 * entries, may be NULL; latency = done_s - arrival_s; the times after
 * arrival are -1 for a request that failed). Results
 * go to an output ring of ring_points int32 that the call allocates and
 * reuses in request order; a request waits for room in it (which then
 * counts in its latency), and none may be longer than the ring
 * (ACT_E_RANGE). The ring is allocated and written once before the first
 * submission (tens of milliseconds for 2^26 points), so the first arrival
 * should lie that far ahead of the call: a request whose arrival time has
 * passed is submitted at once, and the delay counts in its latency.
 * Returns once every request has completed: ACT_OK or the first failure.
 */
int act_server_replay(act_server *s, int64_t n, const int32_t *index,
                      const double *const *h_points, const int64_t *n_points,
                      const double *arrival_s, int64_t ring_points, act_request_times *times);
int act_server_stats_get(act_server *s, act_server_stats *stats);
double act_server_clock(void);
/* Finish every queued request, then release streams and arenas. */
void act_server_destroy(act_server *s);
const char *act_server_last_error(void);

/* Rate of the GPU wall clock used by batch completion ticks. */
int act_wall_clock_hz(int32_t device, double *hz);

/*
 * act_cell_ids -- level-30 cell ids of n points (Section II, S2 paragraph:
 * 3 face bits, a Hilbert-ordered bit pair per level, a marker bit). The
 * projection is lat/lng -> unit sphere -> cube face (u, v) -> linear
 * (s, t) = ((1 + u) / 2, (1 + v) / 2) -> 30-bit (i, j) -> Hilbert
 * position, in fp64. Invalid points get
 * id 0. d_points: device 2*n doubles; d_ids: device n uint64. The points'
 * device must be the current HIP device.
 */
int act_cell_ids(const double *d_points, int64_t n, uint64_t *d_ids,
                 void *stream);

/* Index metrics (the paper's index-metrics table (Table I) analogues plus sizes). */
typedef struct {
  int64_t n_polys;
  int64_t n_edges;
  int64_t n_cells;          /* cells of the super covering                    */
  int64_t n_cells_interior_only; /* cells whose references are all true hits */
  int64_t n_nodes;          /* trie nodes (256 entries each), node 0 reserved */
  int64_t node_bytes;       /* device bytes of the trie (32-bit entries)      */
  int64_t lut_words;        /* uint32 words of the lookup table               */
  int64_t edge_bytes;       /* device polygon store                           */
  int64_t device_bytes;     /* total HBM held by the index                    */
  int32_t max_depth;        /* deepest node level (root = 1)                  */
  int32_t max_refs;         /* most references of one cell                    */
  int32_t max_cell_level;
  int32_t n_faces;          /* faces with a trie                              */
  int32_t face_prefix_level[6]; /* per-face common-prefix level, -1 if none  */
  int32_t mode;
  int32_t lds_nodes;        /* trie nodes staged in LDS (default depth)     */
  double precision_m;
  double build_seconds;
  int64_t local_words;      /* cell-local refinement records (32-bit words)   */
  int64_t train_splits;     /* cells split by training (Section III-D)        */
  int64_t train_points_used; /* training points consumed before the budget
                               ran out (n_train if it did not)               */
  int64_t image_bytes;      /* device bytes the index's image needs (equal to
                               device_bytes once uploaded; also for
                               host-only builds)                            */
  double margin_deg;        /* cell margin used (degrees; SPHERE: widened by
                               the largest arc-to-chord distance)           */
  int32_t geometry;         /* ACT_GEOM_*                                    */
  int32_t reserved;
} act_stats;

int act_index_stats(const act_index *idx, act_stats *out);

/*
 * act_lookup_host -- host-side trie lookup of n leaf cells given as
 * (face, i, j) with 30-bit i, j (inspection and tests): writes the tagged
 * trie entry each ends at (0 = false hit) to entries[i]. Host pointers.
 */
int act_lookup_host(const act_index *idx, const int32_t *face, const uint32_t *i,
                    const uint32_t *j, int64_t n, uint64_t *entries);

/*
 * act_refine_local_host -- evaluate, on the host, the cell-local refinement
 * record of candidate polygon `poly` in the cell of leaf (face, i, j) for
 * the point (lat, lng) (tests): *covered = 1 if the polygon covers the
 * point, 0 otherwise. ACT_E_ARG if `poly` is not a candidate of that cell
 * or the index has no records (approximate mode).
 */
int act_refine_local_host(const act_index *idx, int32_t face, uint32_t i, uint32_t j,
                          double lat, double lng, int32_t poly, int32_t *covered);

/*
 * act_lut_host -- copy of the lookup table (host). If `words` is NULL only
 * *n_words is set. Encoding per list (Section III-C): number of true hits,
 * the true-hit ids, number of candidate hits, the candidate ids; ids sorted
 * ascending within each part. Trie entries with tag 3 hold word offsets.
 */
int act_lut_host(const act_index *idx, uint32_t *words, int64_t *n_words);

/*
 * act_encode_refs_host -- encode one reference list exactly as the builder
 * does (tests): refs[k] = polygon id << 1 | interior flag. Returns the
 * tagged entry in *entry and appends to / reuses the LUT held in `lut`
 * (capacity `lut_cap` words, current length *lut_len) for lists of three or
 * more references.
 */
int act_encode_refs_host(const uint32_t *refs, int32_t n_refs,
                         uint32_t *lut, int64_t lut_cap, int64_t *lut_len,
                         uint64_t *entry);

/*
 * act_orient_fp32_host -- the fp32 refinement tier's decision for one
 * orientation test, evaluated on the host with the same code the GPU runs
 * (tests): translates a, b, p by `origin` (x = lng, y = lat), rounds to
 * fp32, and returns +1 / -1 when the proven error bound decides the sign of
 * (bx-ax)(py-ay) - (by-ay)(px-ax), 0 when it does not. `m_poly` is the
 * largest |translated coordinate| of the polygon (as the builder stores it).
 */
int act_orient_fp32_host(const double *a, const double *b, const double *p,
                         const double *origin, float m_poly);

/* Exact orientation sign as used by the builder and the last refinement
 * tier (host evaluation, tests). */
int act_orient_exact_host(const double *a, const double *b, const double *p);

/* Many orientation tests at once on the host (tests): abp holds n rows
 * (ax, ay, bx, by, px, py) as (x = lng, y = lat). tier 0: out[k] = the exact
 * sign (act_orient_exact_host); tier 1: out[k] = the fp32 tier's decision
 * (act_orient_fp32_host with origin[2k..2k+1] and m_poly[k]). */
int act_orient_host_n(const double *abp, const double *origin, const float *m_poly, int64_t n,
                      int32_t tier, int8_t *out);

/* Message of the last failure on the calling thread ("" if none). */
/*
 * act_abi_sizes -- sizeof(act_build_opts), sizeof(act_join_args) and
 * sizeof(act_stats) in sizes[0..2], for bindings that mirror the structs.
 */
int act_abi_sizes(int64_t *sizes);

const char *act_last_error(void);

/* Library version string. */
const char *act_version(void);

#ifdef __cplusplus
}
#endif

#endif /* ACT_H */
