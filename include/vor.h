/*
 * vor.h -- C ABI of the MI355X projector-algorithm Voronoi/Delaunay library (libvor.so).
 *
 * The library computes, for n distinct integer point sites in an axis-aligned box X (or a convex
 * polygon X), every Voronoi cell of the diagram restricted to X (Section 2, definition of the Voronoi
 * diagram; Section 3, Method 3.1; Section 4, Algorithm 1 with the endpoint method of Section 5
 * and Appendix 1), stored as in Section 6, and the Delaunay graph read off the neighbour lists
 * (Section 7).  Each cell is computed independently of the others (Theorem 9.1(d)).
 *
 * No C++ exception or torch type crosses this boundary.  Every function returns an int status
 * (VOR_OK or a negative VOR_E_* code) unless noted.  Threading: vor_submit / vor_poll are
 * thread-safe; vor_compute and vor_compute_batch serialise per context.
 *
 * Coordinates: int32, |coordinate| <= 2^30, box extent x1-x0 and y1-y0 at most 2^24.
 * X is the box, or a convex polygon given with the set (Remark 11.1 on a general convex X).
 * Sites must lie in the closed X and be pairwise distinct (problem statement in Section 2; a
 * duplicate is an error, never silently dropped, since dropping it would renumber the sites).
 * The problem statement takes the sites in the interior of X and notes that the definition of
 * a cell extends to sites on its boundary: such sites are accepted, and their cells are computed
 * in the box grown by one unit (which holds them strictly inside) and intersected with X, the
 * embedding of the paper's remark on a non-polygonal X (Section 10).
 */
#ifndef VOR_H
#define VOR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------------- */
#define VOR_OK 0
#define VOR_PENDING 1          /* vor_poll: ticket not finished yet                           */
#define VOR_E_INVAL (-1)       /* null pointer, n == 0, empty or inverted box, bad argument   */
#define VOR_E_DOMAIN (-2)      /* a site outside X, |coord| > 2^30, extent > 2^24             */
#define VOR_E_DUPLICATE (-3)   /* two equal sites                                             */
#define VOR_E_NOMEM (-4)       /* device memory or the HBM budget cannot hold the job         */
#define VOR_E_DEVICE (-5)      /* a HIP runtime error                                         */
#define VOR_E_TICKET (-6)      /* unknown or already consumed ticket                          */
#define VOR_E_CAPACITY (-7)    /* a cell with more lines than the deep pass holds (65536)    */

/* ---- side codes used in neighbour lists (Section 6: boundary lines get unique indices) ---- */
#define VOR_SIDE_BOTTOM (-1)   /* y = y0 */
#define VOR_SIDE_RIGHT (-2)    /* x = x1 */
#define VOR_SIDE_TOP (-3)      /* y = y1 */
#define VOR_SIDE_LEFT (-4)     /* x = x0 */
/* Convex polygon X with vertices v_0..v_{K-1} (counter-clockwise): side e runs from v_e to
 * v_{e+1 mod K} and is named -(e+1); its line is N.x <= N.v_e with N = (dy, -dx) / gcd(|dx|, |dy|)
 * for (dx, dy) = v_{e+1} - v_e (the primitive outward normal).  The box is the polygon
 * (x0,y0), (x1,y0), (x1,y1), (x0,y1): the codes above with the same lines. */
#define VOR_MAX_SIDES 256

/* ---- flags ------------------------------------------------------------------------------ */
#define VOR_SET_DEVICE 0x1u       /* vor_set.x / .y are device pointers (HBM-resident input)  */
#define VOR_RESULT_DEVICE 0x2u    /* opts: result arrays stay in device memory (owned by the
                                     context, valid until the next call or vor_result_free)  */
#define VOR_NO_VERTICES 0x4u      /* opts: do not write vertex rationals (vtx == NULL)         */
#define VOR_CHECK_SYMMETRY 0x8u   /* opts: count asymmetric neighbour pairs into stats          */
#define VOR_TIME_KERNELS 0x10u    /* opts: HIP events between the pipeline stages (*_ms fields) */

typedef struct vor_ctx vor_ctx;   /* opaque: device memory pools, streams, request loop */

typedef struct {
    int32_t x0, y0, x1, y1;       /* X = [x0, x1] x [y0, y1] */
} vor_box;

/* One point set in structure-of-arrays form.  Borrowed for the duration of vor_compute*,
 * copied by vor_submit.  With nregion = 0, X is `box`.  With 3 <= nregion <= VOR_MAX_SIDES, X is
 * the convex polygon (region_x[i], region_y[i]) (host memory, counter-clockwise, strictly convex:
 * every turn strictly left, the boundary going round once; VOR_E_INVAL otherwise) and `box` is
 * ignored (the polygon's bounding box, extent at most 2^24, takes its place). */
typedef struct {
    uint32_t n;
    const int32_t *x;
    const int32_t *y;
    vor_box box;
    uint32_t flags;               /* VOR_SET_DEVICE */
    uint32_t nregion;             /* 0, or the number of vertices of a convex polygon X */
    const int32_t *region_x;      /* [nregion] */
    const int32_t *region_y;      /* [nregion] */
} vor_set;

typedef enum {
    VOR_EXACT_ONLY = 0,           /* every predicate in exact integer arithmetic            */
    VOR_FP32_FILTERED = 1         /* FP32 filter with a stated error bound, exact fallback    */
} vor_precision;

typedef struct {
    int device;                   /* HIP device ordinal                                       */
    uint64_t hbm_budget_bytes;    /* admission budget of the request loop (0 = 3/4 of HBM)    */
    int32_t precision;            /* vor_precision                                            */
    uint32_t flags;               /* VOR_RESULT_DEVICE | VOR_NO_VERTICES | VOR_CHECK_SYMMETRY  */
} vor_opts;

/* Vertex in pair form: the point (X/d, Y/d), X and Y two's-complement 128-bit integers split
 * into 64-bit halves, d > 0.  Not reduced by the gcd: X, Y, d are Cramer's rule applied to the
 * two lines N.x <= c of the vertex in absolute coordinates (site line N = 2(p_j - p_k),
 * c = |p_j|^2 - |p_k|^2; sides use their unit outward normal). */
typedef struct {
    uint64_t x_lo;
    int64_t x_hi;
    uint64_t y_lo;
    int64_t y_hi;
    int64_t d;
} vor_rat;

/* Work counters of one call (Theorem 9.1(b): rays, nodes of the algorithm tree and distance
 * comparisons per cell). */
typedef struct {
    uint64_t rays;            /* rays shot (Lemma on shot rays: sum <= 11 n for a rectangle)  */
    uint64_t nodes;           /* subedges classified (Lemma on tree nodes: <= 2 e_k per cell)  */
    uint64_t evals;           /* candidate evaluations ("distance comparisons")              */
    uint64_t exact_decisions; /* predicates the FP32 filter left to exact arithmetic          */
    uint64_t deferred_cells;  /* cells moved from the filtered pass to the exact pass         */
    uint64_t asym_pairs;      /* with VOR_CHECK_SYMMETRY: neighbour pairs seen one way only   */
    uint64_t shells;          /* bucket shells scanned                                        */
    uint64_t edges;           /* sum of e_k                                                   */
    uint64_t vertex_tests;    /* rays towards a candidate vertex that confirmed it            */
    uint64_t adaptive_cells;  /* cells whose scans met a crowded bucket, computed again over
                                 the refined buckets (adaptive bucketing of Method 11.5)      */
    uint64_t adaptive_evals;  /* candidate evaluations of that pass (included in evals)       */
    /* Exact fallbacks by predicate kind (exact_decisions = fallback_cmp + fallback_incircle).
     * A plain ray's decision orders the hit parameters t_j = c_j / (N_j.d) of eq. Tdef; a
     * vertex ray's decision is whether u = L1 ∩ L2 lies in the cell, an incircle-type test
     * (Algorithm 1, lines Vertex / OutsideCell).  Rates: fallback_cmp / (rays + vertex_tests -
     * vertex_rays) and fallback_incircle / vertex_rays.  With VOR_EXACT_ONLY every decision is
     * exact and these count nothing. */
    uint64_t fallback_cmp;      /* plain rays whose FP32 argmin was not certified             */
    uint64_t fallback_incircle; /* vertex rays whose FP32 decision was not certified          */
    uint64_t vertex_rays;       /* rays shot towards a candidate vertex (Den > 0)             */
} vor_stats;

/* Result of one point set.  Host memory owned by the library (device memory with
 * VOR_RESULT_DEVICE) until vor_result_free. */
typedef struct {
    uint32_t n;
    const uint32_t *cell_off;  /* [n+1] CSR offsets into nbr / vtx                            */
    const int32_t *nbr;        /* [cell_off[n]] per cell, CCW, lines that carry an edge of
                                  positive length: site index 0..n-1 or a side code (box:
                                  VOR_SIDE_*, polygon: -(e+1));
                                  rotated so the entry smallest as uint32 comes first         */
    const vor_rat *vtx;        /* [cell_off[n]] vtx[i] = line(nbr[i]) ∩ line(nbr[i+1 cyclic]);
                                  NULL with VOR_NO_VERTICES                                   */
    uint64_t m;                /* Delaunay edges                                              */
    const uint32_t *del;       /* [2m] pairs (i, j), i < j, lexicographically sorted          */
    vor_stats stats;
    float device_ms;           /* device time of the pipeline (HIP events)                     */
    float cells_ms;            /* with VOR_TIME_KERNELS: filtered cell pass                    */
    float exact_ms;            /* with VOR_TIME_KERNELS: exact / deep cell passes              */
    float grid_ms;             /* with VOR_TIME_KERNELS: validation, grid build, refinement    */
    float emit_ms;             /* with VOR_TIME_KERNELS: CSR, vertices, Delaunay edges         */
    int32_t graph_replayed;    /* 1 when the pipeline ran as replayed HIP graph(s)            */
    int32_t status;            /* VOR_OK, or the error of this set inside a batch             */
    float adaptive_ms;         /* with VOR_TIME_KERNELS: the pass over refined buckets         */
    double t_submit, t_admit, t_done; /* request loop: the request's submit / admission / done
                                         times (seconds, monotonic clock); 0 otherwise        */
} vor_result;

/* Create a context on opts->device (NULL opts: device 0, FP32 filtered, host results). */
int vor_create(const vor_opts *opts, vor_ctx **out);

/* Destroy a context: pending tickets are cancelled, their results freed. */
int vor_destroy(vor_ctx *ctx);

/* Blocking: one point set -> *out (free with vor_result_free).  Every cell is computed on its
 * own by the projector (Algorithm 1 with the endpoint method of Section 5 / Appendix 1 over the
 * buckets of Method 11.5), the cells in parallel (Theorem 9.1(d)).  A set holds at most 2^27
 * sites (VOR_E_INVAL beyond): entry offsets are 32-bit, and the entries of n sites in a K-gon
 * number at most 6n + K - 6 (Euler's formula). */
int vor_compute(vor_ctx *ctx, const vor_set *set, vor_result **out);

/* Blocking: k independent point sets in one launch per pipeline stage (the cells of every set
 * of the batch in each kernel's grid, so that the cells of all sets run in parallel as
 * Theorem 9.1(d) allows); a shape's first call launches kernel by kernel, and from its second
 * call on the pipeline runs as a captured HIP graph, replayed while the shape repeats.
 * outs[i] receives set i's result (its status field carries a per-set error: a set with an
 * input error is found by running the sets one by one, and the others still succeed).  The
 * sets together hold at most 2^27 sites (VOR_E_NOMEM beyond, before any device work; split
 * larger batches).  Host inputs only (VOR_SET_DEVICE: VOR_E_INVAL). */
int vor_compute_batch(vor_ctx *ctx, const vor_set *sets, uint32_t k, vor_result **outs);

/* Request loop (the parallel setting of Theorem 9.1(d) applied to independent requests):
 * copy the set into library memory and enqueue it; returns immediately with a ticket.  A host
 * thread admits queued requests in submission order into one of four device workspaces (each
 * admitted group runs as one batched pipeline, as vor_compute_batch) while their HBM
 * footprints (vor_footprint) and those of the batches already on the GPU fit the context's
 * budget; up to four admitted groups overlap on the device.  Thread-safe.  VOR_E_INVAL for a bad set
 * or device input (VOR_SET_DEVICE). */
int vor_submit(vor_ctx *ctx, const vor_set *set, uint64_t *ticket);

/* VOR_OK (and *out, ownership passes to the caller; its t_* fields hold the request's latency
 * stamps), VOR_PENDING, or the request's error (VOR_E_NOMEM: larger than the whole budget).  A
 * ticket is consumed by the poll that returns VOR_OK or an error: the context keeps nothing of
 * it, and later polls of it return VOR_E_TICKET.  Thread-safe. */
int vor_poll(vor_ctx *ctx, uint64_t ticket, vor_result **out);

/* Latency stamps (seconds, monotonic clock) of a ticket not yet consumed: submit, admission
 * (0 while queued), done (0 while running).  VOR_E_TICKET for unknown or consumed tickets. */
int vor_ticket_times(vor_ctx *ctx, uint64_t ticket, double *t_submit, double *t_admit,
                     double *t_done);

/* Number of tickets the context holds (submitted and not yet consumed by vor_poll). */
int vor_ticket_count(vor_ctx *ctx, uint64_t *held);

/* HBM footprint in bytes that admission charges for the set under the context's options and
 * tuning (device buffers of one pipeline run: inputs, grid, refinement, queues, the filtered
 * pass's lines, the entry pool sized by 6n + K + 16, vertices unless VOR_NO_VERTICES, Delaunay
 * pairs).  Errors as vor_compute's validation. */
int vor_footprint(vor_ctx *ctx, const vor_set *set, uint64_t *bytes);

void vor_result_free(vor_result *r);

/* Host copy of a result whose arrays are device memory (VOR_RESULT_DEVICE, or a result struct
 * filled with device pointers of the same layout): n, cell_off, nbr, vtx (may be NULL), m and
 * del are read from `dev`, the arrays copied, every other field taken over.  The device arrays
 * must still be valid (before the context's next call).  *out is host memory owned by the
 * library until vor_result_free.  VOR_E_INVAL for null arguments, VOR_E_DEVICE on a copy error.
 * (Section 6 representation and Section 7 Delaunay list, as vor_compute returns them.) */
int vor_result_to_host(vor_ctx *ctx, const vor_result *dev, vor_result **out);

/* Where k results keep their host arrays, in one call: for bindings that wrap many results at
 * once (a batch's results share one library block).  Row i of `table` (8 words) describes
 * results[i]: n, m, the addresses of cell_off, nbr, vtx (0 when NULL) and del, then the address
 * and byte size of the library block that holds those arrays (0 and 0 when they are not in one
 * such block, as for device results or a result with an error status).  A NULL results[i]
 * gives a row of zeros.  Nothing is modified or freed.  VOR_E_INVAL for a NULL argument. */
int vor_result_layout(const vor_result *const *results, uint32_t k, uint64_t *table);

/* Static string for a status code (never NULL). */
const char *vor_strerror(int status);

/* Tuning knobs (chosen by the autotuner).  sites_per_bucket: target mean bucket occupancy
 * of the uniform grid (Method 11.5); block: threads per workgroup of the cell kernel
 * (64, 128 or 256); block_halfwidth: h, the cell's (2h+1)^2 bucket block scanned before
 * further shells (1..16, 0 = round(2 / sqrt(sites_per_bucket))); leaf_halfwidth: leaf sides
 * around p's leaf bucket that the coordinate-rectangle scan takes first (0..4); scan_path:
 * VOR_PATH_GRID_FIRST (bucket-rectangle scans, cells that meet a crowded bucket move to the
 * coordinate-rectangle scan over the refined buckets) or VOR_PATH_TREE (every cell through the
 * coordinate-rectangle scan).  Results do not depend on any knob.  A new context starts with
 * {1.5, 256, 2, 0, VOR_PATH_GRID_FIRST}, or {1.0, 256, 1, 0, VOR_PATH_GRID_FIRST} with
 * VOR_EXACT_ONLY. */
#define VOR_PATH_GRID_FIRST 0
#define VOR_PATH_TREE 1
typedef struct {
    float sites_per_bucket;
    int32_t block;
    int32_t block_halfwidth;
    int32_t leaf_halfwidth;
    int32_t scan_path;
} vor_tuning;

int vor_set_tuning(vor_ctx *ctx, const vor_tuning *t);
int vor_get_tuning(vor_ctx *ctx, vor_tuning *t);

/* Per-set grid parameters by size class, for batches and the request loop (the autotuner's
 * batch table, Method 11.5's bucket side and the warm-start block of Method 11.6 per set):
 * a set of n sites takes sites_per_bucket, block_halfwidth and leaf_halfwidth from the entry
 * whose log2n is nearest to log2(n) (the first on a tie); block and scan_path stay the context's
 * (they are launch-wide).  count == 0 clears the table (every set uses vor_set_tuning's).  At
 * most 64 entries; ranges as vor_tuning, 0 <= log2n <= 30; VOR_E_INVAL otherwise.  Results do
 * not depend on it. */
typedef struct {
    int32_t log2n;
    float sites_per_bucket;
    int32_t block_halfwidth;
    int32_t leaf_halfwidth;
} vor_size_tuning;
int vor_set_size_tuning(vor_ctx *ctx, const vor_size_tuning *t, uint32_t count);

/* Lloyd iterations on the integer grid (centroidal Voronoi relaxation, the kind of repeated
 * diagram computation the paper's introduction motivates the method with).  Each of `iters`
 * steps computes the diagram of the current sites (X and validation as vor_compute) and moves
 * every site to the rounded centroid of its cell:
 *   the cell's vertices relative to its site p in IEEE double, u_t = fl(X_t - p D_t) / fl(D_t)
 *   (exact integer, correctly rounded conversion); c_t = u_t.x u_{t+1}.y - u_{t+1}.x u_t.y;
 *   A2 = sum c_t, S = sum (u_t + u_{t+1}) c_t in the stored order from t = 0 (every operation
 *   rounded once); proposal = p + rint(S / (3 A2)) (half to even), or p when that point is not
 *   strictly inside X; then, while a position is proposed by more than one site, every such
 *   site whose proposal is not its current position keeps its current position.
 * set: host arrays only (VOR_SET_DEVICE: VOR_E_INVAL).  out_x, out_y: [n] host arrays, the sites
 * after the last step (same ids).  moved: NULL or [iters] host array, the number of sites that
 * moved in each step.  Errors as vor_compute. */
int vor_lloyd(vor_ctx *ctx, const vor_set *set, uint32_t iters, int32_t *out_x, int32_t *out_y,
              uint32_t *moved);

/* Diagnostic (not on the hot path): the FP32 filter keys that the cell passes compute for one
 * line and one ray direction each, so that their bounds can be checked in exact arithmetic
 * (the filter sits in front of the exact comparisons of eq. Tdef, Theorem 2.2; buckets and
 * filtered candidate scans of Method 11.5).  Frame: p-relative and doubled, a line is
 * N.w <= c with N = (nx[i], ny[i]).
 *   kind[i]  0: site candidate, N = delta = a - p, c = |delta|^2 (c[i] ignored);
 *            1: general line with c = c[i], 0 < c <= 2^50 (box sides are such lines)
 *   nx, ny   |.| <= 2^24, not both zero
 *   dir      [4n] ray direction d as two signed 128-bit integers, each given as
 *            (high 64 bits, low 64 bits): x_hi, x_lo, y_hi, y_lo; |component| < 2^100
 *            (|high| < 2^36), d != 0
 *   out      [8n] floats per instance: key_lo, key_hi, key_lo * (1 - 2^-19),
 *            key_hi * (1 + 2^-19), upper bound of the exact endpoint parameter (as used after an
 *            exact decision; +inf when N.d <= 0), d_s.x, d_s.y, 0.  Keys are in units of
 *            d_s = d 2^-sigma: the exact key is c 2^sigma / (N.d) when N.d > 0.
 *   sigma    [n] the scaling exponent
 * All arrays are host memory owned by the caller; n == 0 is a no-op.  Returns VOR_E_INVAL for
 * a null pointer or an argument out of range, VOR_E_NOMEM / VOR_E_DEVICE for HIP failures. */
int vor_filter_keys(int32_t device, int64_t n, const int32_t *kind, const int32_t *nx,
                    const int32_t *ny, const int64_t *c, const int64_t *dir, float *out,
                    int32_t *sigma);

/* Diagnostic (not on the hot path): the candidate regions that the scans certify for one ray
 * bound, computed by the same device functions the cell passes use, so that they can be checked
 * in exact arithmetic against the lemma on sites in the large square (Appendix 1: every site
 * not farther from y than p lies in the square S[y, |y - p|], hence in the integer rectangle of
 * eq. (S_I)) for the point y = p + (T/2) d_s of Method 11.6.  Frame: coordinates relative to
 * the box origin; the ray parameter is doubled (w = 2 (x - p) = t d_s).
 *   geom    [7n] per instance: px, py (0 <= p <= extent), W, H (box extent, 1..2^24), s
 *           (bucket side >= 1), gx, gy (grid, gx s >= W, gy s >= H)
 *   dir     [4n] ray direction d as in vor_filter_keys (|component| < 2^100, d != 0)
 *   T       [n] upper bound of the endpoint parameter in units of d_s = d 2^-sigma
 *           (>= 0; +inf: the whole region)
 *   z       [2n] one test point per instance (relative coordinates, |.| <= 2^25)
 *   rects   [8n] out: the bucket rectangle bx0, bx1, by0, by1 (inclusive, clipped to the grid),
 *           then the coordinate rectangle x0, x1, y0, y1 (inclusive, clipped to the box)
 *   disk    [3n] out: centre (p-relative) and squared radius of the pruning disk
 *   inside  [n] out: 1 when the disk test admits z
 *   sigma   [n] out: the scaling exponent;  ds [2n] out: d_s as the scans round it
 * Host arrays owned by the caller; n == 0 is a no-op.  VOR_E_INVAL for a null pointer or an
 * argument out of range, VOR_E_NOMEM / VOR_E_DEVICE for HIP failures. */
int vor_region_diag(int32_t device, int64_t n, const int32_t *geom, const int64_t *dir,
                    const float *T, const int32_t *z, int32_t *rects, float *disk,
                    int32_t *inside, int32_t *sigma, float *ds);

/* Measured peaks of GPU `device`, for roofline figures beside the published ones (diagnostics,
 * not part of the Voronoi computation; each call allocates and frees its own device buffers and
 * runs on a stream of its own, so it takes a few milliseconds).
 *   vor_peak_fp32: FP32 FMA rate in TFLOP/s (2 flops per FMA) of a register-only loop built like
 *                  the cell kernels, without packed FP32 instructions.
 *   vor_peak_copy: device-to-device copy of `bytes` (rounded down to 16-byte words, at least 16)
 *                  in GB/s, bytes read plus bytes written.
 * Both return VOR_OK, VOR_E_INVAL (null output, bytes < 16), VOR_E_NOMEM or VOR_E_DEVICE. */
int vor_peak_fp32(int32_t device, double *tflops);
int vor_peak_copy(int32_t device, uint64_t bytes, double *gbps);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): vor_compute of one set that allocates nothing.  Every
 * working buffer of the run is carved out of a fixed device array of the library,
 * VOR_NOALLOC_SCRATCH_BYTES on each GPU it runs on (held until the process ends); the outputs go
 * to the caller's device buffers.  No hipMalloc, hipFree or other allocating call is made.
 *   device     GPU ordinal
 *   stream     hipStream_t the work is enqueued on (NULL: the null stream); the call returns
 *              after that stream has finished the call's work
 *   set        n <= VOR_NOALLOC_MAX_SITES; x, y device pointers (VOR_SET_DEVICE) or host
 *              arrays; the box or a convex polygon X as for vor_compute
 *   precision  vor_precision; tuning: the defaults of a new context
 *   cell_off   [n+1] device: CSR offsets (as vor_result.cell_off)
 *   nbr        [nbr_cap] device: neighbour lists; nbr_cap >= 6n + K + 16 (K = 4 for the box)
 *   vtx        [nbr_cap] device: pair-form vertices, or NULL (no vertices)
 *   del        [2 del_cap] device: Delaunay pairs; del_cap >= 3n + 8
 *   entries, m host out: cell_off[n] and the number of Delaunay pairs;  stats: host out or NULL
 * Every call on a GPU shares that GPU's array, which keeps the last call's contents (the run
 * clears what must start at zero itself).  Calls of one process on one GPU are serialised by a
 * lock held until the call's work is done; work the caller enqueues elsewhere that touches the
 * outputs must wait for the return.  VOR_E_INVAL for n above the maximum, capacities below the
 * bounds, null pointers or a bad set; validation and device errors as vor_compute. */
#define VOR_NOALLOC_MAX_SITES 32768u
#define VOR_NOALLOC_SCRATCH_BYTES (32u << 20)
int vor_compute_noalloc(int32_t device, void *stream, const vor_set *set, int32_t precision,
                        uint32_t *cell_off, int32_t *nbr, vor_rat *vtx, uint64_t nbr_cap,
                        uint32_t *del, uint64_t del_cap, uint64_t *entries, uint64_t *m,
                        vor_stats *stats);

/* Version string of the library build (never NULL). */
const char *vor_version(void);

#ifdef __cplusplus
}
#endif
#endif /* VOR_H */
