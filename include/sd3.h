/*
 * sd3 -- exact 3D distance and 3D intersects between triangulated surfaces
 * (TINs, polyhedral surfaces) on AMD Instinct MI355X (gfx950).
 *
 * The two operators are those of "Full Speed Ahead: 3D Spatial Database
 * Acceleration with GPUs" (arXiv 1808.09571):
 *   - 3D Distance (Sec. 3.2.2): per-face distances between the two geometries
 *     followed by the minimum, which is returned to the caller; each per-face
 *     distance minimises the squared distance Q of Eq. 3 over closed parameter
 *     ranges.
 *   - 3D Intersection (Sec. 3.2.3): per-face segment/plane crossing followed by
 *     the barycentric inside test of Eq. 4, with closed constraints (touching
 *     counts as intersecting).
 * Both are generalised from the paper's segment/triangle primitive to
 * triangle/triangle pairs (edge/edge, vertex/face and edge/face-crossing
 * tests) so that two meshes can be compared.  A geometry is the union of its
 * closed triangles (surface semantics: a mesh nested inside a closed mesh
 * does not intersect it).
 *
 * Results: distance is the Euclidean distance in FP64 (0 when the geometries
 * intersect, +inf when either is empty); intersects is exact (decided with
 * exact orientation signs).  The bulk of the work runs in FP32 with forward
 * error bounds; every pair that the bounds cannot settle is recomputed in
 * FP64, so the returned distance is the FP64 minimum.
 *
 * Batches: row g of the first batch is compared with row g of the second (one
 * geometry pair per table row, Sec. 3.1 "whole column" processing).
 *
 * Thread safety: a context may be used by one host thread at a time.  Calls are
 * synchronous (they return after the results are in `out`), except graph
 * launches (sd3_graph_launch).
 */
#ifndef SD3_H
#define SD3_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum sd3_status {
    SD3_OK = 0,
    SD3_E_INVALID_ARG = 1, /* null pointer, count < 0, mismatched batch sizes,
                              offsets not starting at 0 or decreasing, unknown
                              option value, geometry memory kinds differ */
    SD3_E_INDEX_RANGE = 2, /* a triangle index outside its row's vertices */
    SD3_E_NONFINITE = 3,   /* a NaN or infinite coordinate */
    SD3_E_RANGE = 4,       /* a nonzero |coordinate| outside [2^-256, 2^256]
                              (needed for exact orientation signs) */
    SD3_E_NOMEM = 5,       /* device allocation failed */
    SD3_E_DEVICE = 6,      /* HIP runtime error; see sd3_last_error() */
    SD3_E_NO_DEVICE = 7,   /* no usable gfx950 device */
    SD3_E_CAPACITY = 8     /* an internal work list overflowed its bound */
} sd3_status;

/* Where xyz / tri live.  Offsets are always host memory. */
#define SD3_MEM_HOST 0
#define SD3_MEM_DEVICE 1

/*
 * A batch of `count` triangle meshes in CSR form (one mesh per table row).
 *   xyz   : [v_off[count] * 3] doubles, x y z of every vertex, rows back to back
 *   tri   : [t_off[count] * 3] int32, vertex indices of every triangle, local to
 *           its row (0 <= index < v_off[g+1] - v_off[g])
 *   v_off : [count + 1] int64 host array, v_off[0] = 0, non-decreasing
 *   t_off : [count + 1] int64 host array, t_off[0] = 0, non-decreasing
 *   mem   : SD3_MEM_HOST or SD3_MEM_DEVICE for xyz and tri
 * The caller owns every array; the library keeps no pointer after a call.
 */
typedef struct sd3_geoms {
    const double *xyz;
    const int32_t *tri;
    const int64_t *v_off;
    const int64_t *t_off;
    int64_t count;
    int32_t mem;
} sd3_geoms;

/* Arithmetic of the bulk triangle-pair pass. */
#define SD3_PREC_FP32_RESCUE 0 /* FP32 with error bounds + FP64 rescue (default) */
#define SD3_PREC_FP64 1        /* plain FP64 for every tested pair */

/*
 * Seed round of sd3_distance (results never depend on it): before the main
 * pass, each row's best-ranked candidate tile pair is evaluated, so that its
 * distance tightens the upper bound used to prune the others.
 */
#define SD3_ORDER_BOUND 0   /* rank by bounding-box lower bound (default) */
#define SD3_ORDER_NONE 1    /* no seed round */
#define SD3_ORDER_LEARNED 2 /* rank by the tile-pair ranker MLP (opts.ranker) */

/* Tile-pair ranker MLP: 10 -> 64 -> 64 -> 64 -> 1, ReLU, FP32, parameters
 * packed as W1[64][10] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] w4[64] b4. */
#define SD3_MLP_NIN 10
#define SD3_MLP_NHID 64
#define SD3_MLP_NPARAM 9089
/* One training-log record: 10 features, target, row (int32 bits). */
#define SD3_LOG_STRIDE 12

typedef struct sd3_opts {
    int32_t precision;   /* SD3_PREC_* */
    int32_t order;       /* SD3_ORDER_* */
    int32_t timing;      /* nonzero: record HIP events around each phase on the
                            call's stream and report their durations in stats */
    int32_t tile;        /* triangles per tile: SD3_TILE_32/64/128, or
                            SD3_TILE_AUTO (0): the size sd3_autotune chose for
                            this kind of workload on this context, else 64 */
    const float *ranker; /* device, SD3_MLP_NPARAM floats (SD3_ORDER_LEARNED) */
    float *log;          /* device or NULL: one record per tile pair dequeued by
                            sd3_distance, SD3_LOG_STRIDE floats each */
    int64_t log_cap;     /* records `log` can hold; extra records are dropped */
    int64_t queue_cap;   /* tile pairs the candidate queue holds per pass (0: 2^29);
                            larger workloads are processed in several passes */
    int64_t rescue_cap;  /* 0, or a smaller bound of the FP32 rescue list (2^24) */
    int64_t exact_cap;   /* 0, or the starting bound of the exact-arithmetic list
                            (2^22) */
    int32_t semantics;   /* SD3_SURFACE (default) or SD3_SOLID */
    int32_t reserved32;
} sd3_opts;

/*
 * What a row's mesh stands for.  SD3_SURFACE: the union of its closed
 * triangles (a mesh nested inside a closed mesh does not meet it).  SD3_SOLID:
 * the closed region a closed, consistently oriented, connected mesh bounds
 * (the paper's ore bodies, Sec. 4): two rows meet when their surfaces meet or
 * a vertex of one lies inside the other solid (exact ray parity); the
 * distance is then 0, otherwise the surface distance.  The meshes are not
 * checked for being closed.  Eager calls only (graphs: SD3_E_INVALID_ARG).
 */
#define SD3_SURFACE 0
#define SD3_SOLID 1

#define SD3_TILE_AUTO 0
#define SD3_TILE_32 32
#define SD3_TILE_64 64
#define SD3_TILE_128 128

/* Operator of a graph or a tuning run. */
#define SD3_KIND_DISTANCE 0
#define SD3_KIND_INTERSECTS 1

/* Work counters of the last call (all tile and triangle counts summed over rows). */
typedef struct sd3_stats {
    int64_t tile_pairs_total;     /* sum of tilesA * tilesB */
    int64_t tile_pairs_candidate; /* kept by the bounding-box filter */
    int64_t tile_pairs_evaluated; /* candidates still live when dequeued */
    int64_t tri_pairs_boxed;      /* triangle pairs whose boxes were compared */
    int64_t tri_pairs_fp32;       /* triangle pairs through the FP32 test */
    int64_t tri_pairs_fp64;       /* triangle pairs through the FP64 test */
    int64_t rescued;              /* FP32 pairs sent to the FP64 pass */
    int64_t exact;                /* pairs settled by exact arithmetic */
    double ms_total;              /* wall time of the call, host clock */
    /* with opts.timing: device time of each phase (HIP events on the stream):
       [0] validation + upload, [1] sort + tiles, [2] bounds + queue,
       [3] triangle-pair pass, [4] FP64 rescue, [5] exact arithmetic,
       [6] final reduction and download (FP32 calls of at most 64 rows run the
       rescue inside the exact-arithmetic launch: timed in [5]) */
    double ms_phase[7];
    int64_t logged;                /* training-log records produced (may exceed log_cap) */
    /* with opts.timing: device time summed over the launches of selected
       kernels, and their launch counts: [0] radix-sort scatter, [1] tile
       building, [2] tile-pair box filter, [3] main triangle-pair pass */
    double ms_kernel[4];
    int64_t n_kernel[4];
    int64_t sort_items;            /* keys per radix pass (both sides) */
    int32_t sort_item_bytes;       /* bytes an item moves through the radix
                                      scatter passes (read and written,
                                      summed over the passes) */
    int32_t sort_passes;
    int32_t tile;                  /* triangles per tile used by the call */
    int32_t queue_passes;          /* candidate-queue passes */
    int64_t queue_skew;            /* consistency check of the tile-pair pass:
                                      evaluated tile pairs whose two tiles name
                                      different rows (0 in a correct run) */
    int32_t fallback;              /* work-list overflows the call recovered
                                      from by computing again: a full rescue
                                      list by the plain FP64 pass (same bits),
                                      a full exact list with a 4x longer one */
    int32_t reserved32;
    int64_t tiles_copied;          /* tiles whose coordinate copies were written
                                      (only tiles of queued tile pairs get them) */
} sd3_stats;

typedef struct sd3_ctx sd3_ctx;

/* Default options: SD3_PREC_FP32_RESCUE, SD3_ORDER_BOUND. */
void sd3_default_opts(sd3_opts *opts);

/* Create a context on HIP device `device` (must be gfx950).  *out receives the
 * handle or NULL on error.  Errors: SD3_E_INVALID_ARG (out is NULL),
 * SD3_E_NO_DEVICE, SD3_E_DEVICE. */
sd3_status sd3_create(sd3_ctx **out, int device);

/* Release the context and its device memory.  NULL is accepted. */
sd3_status sd3_destroy(sd3_ctx *ctx);

/*
 * 3D distance, row by row (Sec. 3.2.2: per-face distances, then the minimum
 * returned to the user).
 *   dist : [count] doubles, distance of row g of a to row g of b
 *   hit  : [count] bytes or NULL; 1 where the rows intersect (exact)
 * dist/hit are device pointers when a->mem == SD3_MEM_DEVICE, host pointers
 * otherwise.  opts and stats may be NULL.  stream is a hipStream_t (NULL: the
 * default stream); the call synchronises it before returning.
 * A work list that overflows does not fail the call: the FP32 rescue list is
 * replaced by the plain FP64 pass (identical results), the exact list is
 * enlarged (up to 2^26 entries); stats->fallback counts such re-runs.
 * On any error the outputs are left untouched.
 */
sd3_status sd3_distance(sd3_ctx *ctx, const sd3_geoms *a, const sd3_geoms *b, double *dist,
                        uint8_t *hit, const sd3_opts *opts, sd3_stats *stats, void *stream);

/*
 * sd3_distance for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * kernels and results (bit for bit), but every device buffer of the call is
 * carved from one static device array of 128 MiB that each GPU holds from the
 * library's load until the process ends, and host staging comes from pinned
 * memory sd3_create allocated.  The call allocates no device or pinned memory
 * and calls no allocating HIP routine (its host bookkeeping uses the C++
 * heap).  The caller passes inputs and outputs as for sd3_distance.
 *   Limits: at most 4096 rows; the call's buffers (sort keys, tiles, a
 *   tile-pair queue of at most 2^21 entries per pass, a rescue list of 2^20
 *   and an exact list of 2^18 entries) must fit in the 128 MiB, which holds
 *   roughly 1e6 triangles in all (host inputs are staged there too).
 *   Errors: those of sd3_distance; SD3_E_CAPACITY (outputs untouched, message
 *   in sd3_last_error) when the call needs more rows or more scratch;
 *   SD3_E_INVALID_ARG for opts->timing (HIP events would be created).
 *   A rescue-list overflow recomputes on the plain FP64 pass as sd3_distance
 *   does, inside the same scratch.
 * Every allocation-free call on one GPU shares that GPU's array and its
 * contents are those of the last call: calls that overlap on one GPU (other
 * host threads, other contexts, unsynchronised streams) race and must not be
 * issued.  Each call clears what it needs before use.
 */
sd3_status sd3_distance_noalloc(sd3_ctx *ctx, const sd3_geoms *a, const sd3_geoms *b, double *dist,
                                uint8_t *hit, const sd3_opts *opts, sd3_stats *stats, void *stream);

/*
 * 3D intersects, row by row (Sec. 3.2.3: per-face crossing tests of Eq. 4,
 * combined with OR).  hit : [count] bytes, 1 where the rows share a point.
 * Memory kinds, stream and error behaviour as for sd3_distance.
 */
sd3_status sd3_intersects(sd3_ctx *ctx, const sd3_geoms *a, const sd3_geoms *b, uint8_t *hit,
                          const sd3_opts *opts, sd3_stats *stats, void *stream);

/*
 * 3D volume of each row (Sec. 3.2.1): the divergence theorem with the field
 * p / 3 (Eq. 1) gives V = 1/6 sum over triangles (u, v, w) of
 * u . ((v - u) x (w - u)) (Eq. 2).  Positive for closed meshes whose triangles
 * are counter-clockwise seen from outside; for other meshes it is that flux
 * sum as written (relative to the origin).  vol: [count] doubles (device
 * memory when g->mem == SD3_MEM_DEVICE, else host).  Computed in
 * double-double (about 100 bits before the final rounding): within 1e-12
 * relative of the exact value unless the faces' terms cancel by more than
 * about 2^50.  An empty row gives 0.  Errors: as sd3_validate for the batch;
 * outputs untouched on error.
 */
sd3_status sd3_volume(sd3_ctx *ctx, const sd3_geoms *g, double *vol, sd3_stats *stats, void *stream);

/*
 * Segments (or points) against one triangle mesh: the workload the paper
 * measures (Sec. 4: drill-hole line segments against an ore-body mesh), with
 * the operators of Sec. 3.2.2 (distance: segment/segment, segment/surface and
 * point/surface distances, then the minimum) and Sec. 3.2.3 (intersection:
 * Eq. 4 with closed constraints), plus the distance-threshold filter of
 * Sec. 4 ("filtering drill holes based on their distance").
 *   op    : SD3_SEG_DISTANCE (dist[i] = distance of segment i to the mesh,
 *           flag[i] = intersects, flag may be NULL), SD3_SEG_INTERSECTS
 *           (flag[i] = intersects) or SD3_SEG_WITHIN (flag[i] = 1 iff the
 *           distance sd3 returns for segment i is <= r; r finite, >= 0)
 *   seg   : [n][2][3] doubles, endpoints P0 P1 of each segment; P0 == P1 is a
 *           point.  A segment is the closed set {P0 + t (P1 - P0), t in [0, 1]}
 *   mesh  : a batch of exactly one row (at most 2^25 - 1 triangles)
 *   seg_mem : SD3_MEM_HOST or SD3_MEM_DEVICE; must equal mesh->mem; the
 *           outputs are in the same kind of memory
 * Results equal those of sd3_distance / sd3_intersects on the segment as the
 * degenerate triangle (P0, P1, P1): FP64 distances, exact flags; an empty mesh
 * gives +inf and 0.  Errors as for sd3_distance (validation of the segment
 * coordinates and of the mesh); outputs untouched on error.  stats: box tests
 * in tri_pairs_boxed, FP64 pair tests in tri_pairs_fp64, exact tests in exact.
 */
#define SD3_SEG_DISTANCE 0
#define SD3_SEG_INTERSECTS 1
#define SD3_SEG_WITHIN 2
sd3_status sd3_segments(sd3_ctx *ctx, int32_t op, const double *seg, int64_t n, int32_t seg_mem,
                        const sd3_geoms *mesh, double r, double *dist, uint8_t *flag,
                        sd3_stats *stats, void *stream);

/*
 * Training of the tile-pair ranker (SD3_ORDER_LEARNED) by the library's own
 * kernels.  All arrays are device memory; calls are asynchronous on `stream`
 * (a hipStream_t, NULL: default stream).
 *   x    : [n][SD3_MLP_NIN] features (as logged by sd3_distance)
 *   t, y : [n] targets / outputs
 *   params, grad, m, v : [SD3_MLP_NPARAM] (packed layout above)
 * sd3_mlp_forward:   y = MLP(x).
 * sd3_mlp_loss_grad: *loss = mean((MLP(x) - t)^2) (one device float) and its
 *                    gradient with respect to params (grad is overwritten).
 * sd3_adam_step:     one Adam update (bias-corrected, step >= 1) of `count`
 *                    parameters p with gradient g and moments m, v.
 * Errors: SD3_E_INVALID_ARG for NULL pointers, n < 0, step < 1; SD3_E_NOMEM.
 */
sd3_status sd3_mlp_forward(sd3_ctx *ctx, const float *params, const float *x, int64_t n, float *y,
                           void *stream);
sd3_status sd3_mlp_loss_grad(sd3_ctx *ctx, const float *params, const float *x, const float *t,
                             int64_t n, float *loss, float *grad, void *stream);
sd3_status sd3_adam_step(sd3_ctx *ctx, float *p, const float *g, float *m, float *v, int64_t count,
                         int32_t step, float lr, float beta1, float beta2, float eps, void *stream);

/*
 * The scorer of the learned seed round (SD3_ORDER_LEARNED) applied to given
 * feature rows: y[i] = MLP(x[i]) for x [n][SD3_MLP_NIN], computed by the same
 * device function and LDS weight layout that ranks queued tile pairs inside
 * sd3_distance (one wave per row, lane = hidden unit).  sd3_mlp_forward is the
 * training path's batched forward pass; both evaluate the same network.
 * Device arrays, asynchronous on `stream`.  Errors: SD3_E_INVALID_ARG for NULL
 * pointers or n < 0.
 */
sd3_status sd3_mlp_score(sd3_ctx *ctx, const float *params, const float *x, int64_t n, float *y,
                         void *stream);

/*
 * Batched replay through a HIP graph.  sd3_graph_create plans one call of
 * `kind` (SD3_KIND_DISTANCE: dist and optional hit; SD3_KIND_INTERSECTS: hit)
 * over device-resident batches (mem == SD3_MEM_DEVICE) and records every
 * kernel of it -- validation, sort and tiles, bounds and queue, the
 * persistent triangle-pair pass over all rows, rescue, exact arithmetic, final
 * reduction -- into one graph with its own device work space, so that a
 * launch costs one graph launch and no host synchronisation.
 *   - The batch shapes (offsets, counts), the device pointers and the options
 *     are fixed at creation; the contents of xyz / tri / ranker may change
 *     between launches.  The offsets are copied at creation.
 *   - The contents are validated at creation (errors as for sd3_distance) and
 *     again on the device by every launch: a launch over invalid contents, or
 *     one whose work lists overflow, leaves the outputs untouched and
 *     sd3_graph_result reports the error.  Vertex indices are clamped into
 *     their row before use, so invalid contents never address other memory.
 *   - opts.timing and opts.log are not supported (SD3_E_INVALID_ARG).
 *   - The graph keeps `ctx` (for its device) and must be destroyed before it.
 * sd3_graph_launch enqueues one replay on `stream` (hipStream_t, NULL: the
 * default stream) and returns at once.  sd3_graph_result waits for `stream`
 * and returns the status of the last replay enqueued on it (stats may be
 * NULL; timing fields are zero).  Launches of one graph must not overlap:
 * they share its work space.  Different graphs own different work spaces and
 * may replay concurrently on different streams.
 */
typedef struct sd3_graph sd3_graph;
sd3_status sd3_graph_create(sd3_ctx *ctx, int32_t kind, const sd3_geoms *a, const sd3_geoms *b,
                            double *dist, uint8_t *hit, const sd3_opts *opts, sd3_graph **out);
sd3_status sd3_graph_launch(sd3_graph *graph, void *stream);
sd3_status sd3_graph_result(sd3_graph *graph, sd3_stats *stats, void *stream);
sd3_status sd3_graph_destroy(sd3_graph *graph);

/*
 * Tile-size autotuner.  Runs the call `kind` on the given batches with each
 * candidate tile size (32, 64, 128 triangles): one untimed round, then reps
 * rounds that time the sizes in turn; keeps each size's median wall time of
 * those rounds, and records the fastest size in ctx
 * for this kind of workload (operator, precision, order, and the binary
 * magnitudes of the row count and of the mean triangles per row): later calls
 * with opts->tile == SD3_TILE_AUTO on a workload of the same kind use it.
 * Results do not depend on the tile size.  report may be NULL.
 * Errors: those of sd3_distance / sd3_intersects; reps < 1 is
 * SD3_E_INVALID_ARG.
 */
typedef struct sd3_tune_report {
    int32_t n;       /* candidates timed */
    int32_t best;    /* tile size chosen */
    int32_t tile[4]; /* candidate tile sizes */
    double ms[4];    /* median wall time of one call for each candidate */
} sd3_tune_report;
sd3_status sd3_autotune(sd3_ctx *ctx, int32_t kind, const sd3_geoms *a, const sd3_geoms *b,
                        const sd3_opts *opts, int32_t reps, sd3_tune_report *report, void *stream);

/* Host-side validation of a batch whose xyz/tri are host memory (the checks
 * the two operators run before any launch); needs no device. */
sd3_status sd3_validate(const sd3_geoms *g);

/* Static description of a status code. */
const char *sd3_status_string(sd3_status s);

/* Message of the last error raised on ctx ("" if none). */
const char *sd3_last_error(const sd3_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* SD3_H */
