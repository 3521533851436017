/*
 * mapper_gpu.h -- C ABI of the MI355X mapper library (libmapper_gpu.so).
 *
 * The library computes the mapper graph of Singh, Memoli and Carlsson as used
 * by Zhou et al., "Mapper Interactive" (Background section): given a point
 * cloud X in R^d, a filter (lens) f : X -> R or R^2, a cover of f(X) by n
 * intervals per axis with fractional overlap p, and DBSCAN (Ester et al.)
 * parameters eps and minPts, it clusters each pullback set f^{-1}(V_k) with
 * the Euclidean metric and returns the 1-D nerve of the clusters: one node per
 * cluster, one edge per pair of clusters that share a point.
 *
 * The parameter set mirrors the paper's command-line API (Implementation
 * section: number of intervals, overlap, DBSCAN parameters); 2-D covers take
 * per-axis (n, p) as in the breast-cancer use case.
 *
 * Conventions for every call:
 *   - no C++ exception crosses this boundary; every fallible call returns a
 *     mapper_status, and on failure mapper_last_error() describes it;
 *   - pointers documented as "device" are HIP device pointers on the
 *     context's device; "host" pointers are ordinary process memory;
 *   - the caller keeps ownership of every buffer it passes in; the library
 *     copies what it keeps (clouds, lens directions, lens values);
 *   - all device memory the library uses comes from the caller's arena
 *     (mapper_context_create); it never calls hipMalloc itself;
 *   - all device work is issued on the caller's stream(s).
 *
 * Exactness: the returned graph is identical, bit for bit, to the one defined
 * by the following readings (the paper leaves these points open):
 *   lens        canonical FP64 values: column x_c; L-inf max|x_j|; L2 the
 *               correctly rounded sqrt of sum_j x_j^2 accumulated in order in
 *               FP64; projection sum_j x_j v_j accumulated in order in FP64;
 *   cover       L = (M-m)/(n-(n-1)p), s = L(1-p), lo_k = m + k s,
 *               hi_k = lo_k + L, hi_{n-1} = M, closed intervals, FP64;
 *   distance    D(x,y) = fma chain over j of (x_j - y_j)^2 in FP64, in order;
 *               neighbours iff D <= fl(eps*eps); a point neighbours itself;
 *   DBSCAN      core iff #neighbours >= minPts; clusters = connected
 *               components of core points; a non-core point with core
 *               neighbours joins the lowest-numbered adjacent cluster, else it
 *               is noise (dropped);
 *   labelling   clusters of an element numbered by their smallest core index;
 *               nodes ordered by (element, cluster); element id k1*n2 + k2 in
 *               2-D; members ascending; edges (a<b) lexicographic; weight =
 *               number of shared points.
 * Distance tiles may run in BF16/FP16 on the matrix cores; every pair whose
 * tile distance lies within a rigorous error band of eps^2 is re-decided with
 * the FP64 distance above, so the precision never changes the graph.
 */
#ifndef MAPPER_GPU_H
#define MAPPER_GPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MAPPER_OK = 0,
    MAPPER_EINVAL = -1,     /* invalid argument; nothing was launched */
    MAPPER_ENOMEM = -2,     /* the arena cannot hold the run's workspace */
    MAPPER_EDEVICE = -3,    /* a HIP call failed */
    MAPPER_EBUSY = -4,      /* object still in use (e.g. cloud with requests in flight) */
    MAPPER_ETIMEDOUT = -5,  /* mapper_wait timed out; the request keeps running */
    MAPPER_ENOTIMPL = -6
} mapper_status;

typedef enum {
    MAPPER_LENS_COLUMN = 0,      /* f(x) = x_column */
    MAPPER_LENS_L2 = 1,          /* f(x) = ||x||_2 */
    MAPPER_LENS_LINF = 2,        /* f(x) = max_j |x_j| */
    MAPPER_LENS_PROJECTION = 3,  /* f(x) = <x, direction> */
    MAPPER_LENS_VALUES = 4,      /* f given per point */
    /* Whole-cloud lenses (the density and eccentricity filters the paper
     * lists, Background and Design sections), exact in FP64: */
    MAPPER_LENS_KNN_DISTANCE = 5,  /* f(x) = distance to the k-th nearest other point,
                                      k = the axis' column field (1..16); small where the
                                      cloud is dense (see mapper_knn_d2) */
    MAPPER_LENS_ECCENTRICITY = 6   /* f(x) = largest distance to another point
                                      (L-infinity eccentricity) */
} mapper_lens_kind;

typedef enum {
    MAPPER_PREC_FP32 = 0,    /* FP32 matrix-core tiles */
    MAPPER_PREC_BF16 = 1,    /* one BF16 product per pair, FP32 accumulate */
    MAPPER_PREC_BF16X3 = 2,  /* BF16 hi/lo split, three products */
    MAPPER_PREC_FP16 = 3,    /* one FP16 product per pair */
    MAPPER_PREC_FP16X3 = 4,  /* FP16 hi/lo split, three products */
    MAPPER_PREC_AUTO = 5     /* chosen per run by the tile autotuner */
} mapper_precision;

/* One lens axis and its cover (Background section: filter f, number of
 * intervals n, overlap p). */
typedef struct {
    int32_t kind;            /* mapper_lens_kind */
    int32_t column;          /* COLUMN: 0 <= column < d; KNN_DISTANCE: k */
    const float *direction;  /* PROJECTION: d floats, host; copied */
    const double *values;    /* VALUES: n doubles, host; copied; finite */
    int32_t n_intervals;     /* >= 1 */
    double overlap;          /* 0 <= overlap < 1 */
    int32_t cover;           /* MAPPER_COVER_UNIFORM or MAPPER_COVER_BALANCED */
} mapper_axis;

/* Cover of one lens axis (Background section).  UNIFORM: n closed intervals
 * of equal length tiling [min f, max f], neighbours sharing the fraction p of
 * their length.  BALANCED: intervals holding equal numbers of points (the
 * balanced cover the paper mentions): the uniform cover laid on the rank
 * axis [0, N-1] of the sorted lens values v_0 <= ... <= v_{N-1}, each rank
 * interval [a, b] becoming the closed value interval [v[floor a], v[ceil b]];
 * with distinct values every interval holds between floor(L) + 1 and
 * ceil(L) + 2 points, L = (N-1) / (n - (n-1) p). */
#define MAPPER_COVER_UNIFORM 0
#define MAPPER_COVER_BALANCED 1

typedef struct {
    int32_t n_axes;          /* 1 (1-D mapper) or 2 (2-D mapper) */
    mapper_axis axis[2];
    double eps;              /* DBSCAN eps, finite, >= 0 */
    int32_t min_pts;         /* DBSCAN minPts, >= 1 */
    int32_t precision;       /* mapper_precision */
    uint32_t flags;          /* MAPPER_FLAG_* */
} mapper_params;

#define MAPPER_FLAG_DEBUG_STAGES 1u   /* keep per-stage arrays in the graph */
/* Launch form of the distance tiles (the graph is the same in every form).
 * By default the library picks one: tile pairs (one workgroup per 128 x 128
 * tile pair) when the tile pairs are screened (MAPPER_FLAG_NO_SCREEN below),
 * else macro tiles (one workgroup per pair of 256-row blocks, up to four
 * tile pairs) for single 16-bit products and tile pairs otherwise.  These
 * flags force a form; MACRO (which turns screening off) applies to
 * MAPPER_PREC_BF16/FP16 and to AUTO when it picks one of them, and is
 * ignored otherwise. */
#define MAPPER_FLAG_TILE_PAIRS 2u
#define MAPPER_FLAG_TILE_MACRO 4u
/* Compute every tile pair of every element.  By default a tile pair none of
 * whose rows' landmark cells lies within eps of a cell of its columns (each
 * cell bounded by a ball) is proven to hold no neighbour pair and skipped
 * (clouds of at least 1024 points and d <= 2048, whose members are laid out
 * by cell); the graph is the same. */
#define MAPPER_FLAG_NO_SCREEN 8u

typedef struct mapper_context mapper_context;
typedef struct mapper_cloud mapper_cloud;
typedef struct mapper_graph mapper_graph;

typedef struct {
    double ms_total, ms_lens, ms_bin, ms_tiles, ms_recheck, ms_cc, ms_edges;
    int64_t n_slots;         /* sum over elements of |f^{-1}(V_k)| */
    int64_t pairs;           /* unordered in-element pairs, self included */
    int64_t tiles;           /* tile pairs launched */
    int64_t band_pairs;      /* pairs re-decided in FP64 */
    int64_t bitmask_bytes;   /* adjacency bitmask written */
    uint64_t arena_peak_bytes;
    int32_t precision;       /* precision actually used */
    int32_t tile_m, tile_n, split_terms;
    int32_t tile_launches;   /* > 1 if the band list had to grow (the band records
                                are collected again; macro tiles are redone) */
    double band_halfwidth;   /* largest FP32 half-width of the eps^2 band */
    uint64_t reserved_bytes; /* workspace reserved in one block after binning */
    uint64_t reserve_overflow_bytes;  /* taken beyond the reservation (a regrown band list) */
    int32_t admission_waits; /* serving: times the request waited for its reservation */
    int32_t tile_passes_redone;  /* serving: tile passes lost to a later shortage */
    int64_t tiles_screened_out;  /* tile pairs proven empty by their balls, not computed */
    int64_t pairs_computed;  /* in-element pairs of the tile pairs computed */
    int32_t tune_sampled;    /* MAPPER_PREC_AUTO: 1 if this run timed the precisions (else a cached choice) */
    int32_t tune_pad;
    double tune_pred_ms[5];  /* ... the predicted tile + recheck ms of each precision (FP32, BF16, BF16X3,
                                FP16, FP16X3); the smallest was chosen */
} mapper_run_stats;

/* --- context ------------------------------------------------------------
 * device: HIP device ordinal.  arena: device buffer of arena_bytes (256-byte
 * aligned) that the library sub-allocates; it stays owned by the caller and
 * must outlive the context.  stream: hipStream_t for all work (NULL = the
 * null stream). */
mapper_status mapper_context_create(int device, void *arena, uint64_t arena_bytes,
                                    void *stream, mapper_context **out);
/* Streams for concurrent requests (mapper_submit): count hipStream_t handles,
 * owned by the caller.  Without this call requests use the context stream. */
mapper_status mapper_context_set_streams(mapper_context *ctx, void *const *streams, int count);
void mapper_context_destroy(mapper_context *ctx);
/* Message for the last failure on this thread (never NULL). */
const char *mapper_last_error(void);
/* Bytes of arena currently in use and the high-water mark. */
mapper_status mapper_context_memory(const mapper_context *ctx, uint64_t *in_use, uint64_t *peak);

/* --- point clouds ---------------------------------------------------------
 * points: n x d float32 row-major, host (points_on_device = 0) or device
 * (= 1).  The cloud is copied into the arena and stays resident until
 * mapper_cloud_destroy.  Non-finite coordinates -> MAPPER_EINVAL. */
mapper_status mapper_cloud_create(mapper_context *ctx, const float *points, int64_t n,
                                  int32_t d, int32_t points_on_device, mapper_cloud **out);
mapper_status mapper_cloud_destroy(mapper_cloud *cloud);   /* MAPPER_EBUSY while in use */

/* --- one mapper graph, synchronous ------------------------------------- */
mapper_status mapper_run(mapper_context *ctx, const mapper_cloud *cloud,
                         const mapper_params *params, mapper_graph **out);

/* --- several eps values in one pass, synchronous ------------------------
 * Interactive recomputation as the DBSCAN parameter changes (Design and
 * Implementation section: the graph is recomputed on the fly as parameters
 * change; the eps-selection module of the CIFAR-10 use case).  out[t]
 * (t < n_eps, 1 <= n_eps <= MAPPER_MAX_EPS_VALUES) receives exactly the graph
 * mapper_run returns with params->eps = eps_list[t]; params->eps itself is
 * not used beyond validation.  Lens, cover, pullback sets, panels and the
 * distance tiles are computed once: each tile pair's Gram values are decided
 * against every eps value, each value getting its own bitmask and counts.
 * eps_list: host, n_eps finite values >= 0, any order.  The graphs are owned
 * by the caller (mapper_graph_destroy each); on error every out[t] is NULL. */
#define MAPPER_MAX_EPS_VALUES 4
mapper_status mapper_run_eps_sweep(mapper_context *ctx, const mapper_cloud *cloud,
                                   const mapper_params *params, const double *eps_list,
                                   int32_t n_eps, mapper_graph **out);

/* --- graphs for several (eps, minPts) pairs from one pass, synchronous -------
 * The same interactive recomputation with minPts free as well: out[t * n_minpts
 * + u] receives exactly the graph mapper_run returns with params->eps =
 * eps_list[t] and params->min_pts = minpts_list[u].  A pair's neighbour
 * count and adjacency do not depend on minPts (DBSCAN's core rule compares
 * the count with it afterwards, Background section), so beyond the single
 * eps sweep only the clusters, border points, nodes and edges are computed
 * per minPts value.  eps_list as for mapper_run_eps_sweep; minpts_list: host,
 * n_minpts values >= 1 (1 <= n_minpts <= MAPPER_MAX_MINPTS_VALUES), any
 * order; out holds n_eps * n_minpts graphs owned by the caller; on error
 * every out[.] is NULL. */
#define MAPPER_MAX_MINPTS_VALUES 16
mapper_status mapper_run_sweep(mapper_context *ctx, const mapper_cloud *cloud, const mapper_params *params,
                               const double *eps_list, int32_t n_eps, const int32_t *minpts_list,
                               int32_t n_minpts, mapper_graph **out);

/* --- k-th nearest-neighbour distances, synchronous -----------------------
 * The eps-selection module of the CIFAR-10 use case (Use Cases section)
 * plots the distribution of every point's distance to its k-th nearest
 * neighbour to choose eps.  out_d2[i] (host, n doubles) = the k-th smallest
 * canonical squared distance D(x_i, x_j) over the other points j != i, ties
 * counted with multiplicity; D is the FP64 chain of the eps tiles (x_j - y_j
 * in FP64, fma in coordinate order), so the result is exact and does not
 * depend on `precision` (a MAPPER_PREC_*, AUTO = FP16), which only sets
 * the matrix-core screening pass.  On a cloud with cells (see
 * MAPPER_FLAG_NO_SCREEN) each pass takes only the 128-row column blocks the
 * cells' distance bounds leave; the result is the same.  1 <= k <= min(16,
 * n - 1).  stats may be NULL; ms_tiles is the two screening passes, tiles
 * the block pairs they took, ms_recheck the FP64 step, band_pairs the
 * candidate pairs it evaluated. */
mapper_status mapper_knn_d2(mapper_context *ctx, const mapper_cloud *cloud, int32_t k,
                            int32_t precision, double *out_d2, mapper_run_stats *stats);

/* --- serving: continuous batching of requests ---------------------------
 * submit returns at once with a ticket; requests are admitted while their
 * workspace fits in the arena and a stream slot is free, and run
 * concurrently.  wait blocks up to timeout_us (< 0: forever) and hands over
 * the graph.  A request's graph never depends on what else runs. */
mapper_status mapper_submit(mapper_context *ctx, const mapper_cloud *cloud,
                            const mapper_params *params, uint64_t *ticket);
mapper_status mapper_wait(mapper_context *ctx, uint64_t ticket, int64_t timeout_us,
                          mapper_graph **out);

/* --- graph (host memory owned by the graph) ---------------------------- */
int64_t mapper_graph_num_nodes(const mapper_graph *g);
int64_t mapper_graph_num_edges(const mapper_graph *g);
const int32_t *mapper_graph_node_element(const mapper_graph *g);  /* N element ids */
const int64_t *mapper_graph_node_offsets(const mapper_graph *g);  /* N+1 */
const int32_t *mapper_graph_node_members(const mapper_graph *g);  /* ascending point ids */
const int32_t *mapper_graph_edges(const mapper_graph *g);         /* 2E: (a,b), a<b, sorted */
const int32_t *mapper_graph_edge_weights(const mapper_graph *g);  /* E shared-point counts */
mapper_status mapper_graph_stats(const mapper_graph *g, mapper_run_stats *out);

/* Per-stage arrays, present when MAPPER_FLAG_DEBUG_STAGES was set.
 * name: "lens" (double, n*n_axes, axis-major), "lo", "hi" (double, endpoints
 * of all axes concatenated), "elem_offsets" (int64, E+1), "elem_members"
 * (int32), "slot_count" (int32), "slot_core" (uint8), "slot_node" (int32).
 * Returns the host pointer and element count, or NULL if absent. */
const void *mapper_graph_stage(const mapper_graph *g, const char *name, int64_t *count);
void mapper_graph_destroy(mapper_graph *g);

/* --- test hook -------------------------------------------------------------
 * Gram values of the distance tiles: for the rows `rows` (host, nrows point
 * ids of the cloud) runs the tile kernel of the given precision on them as one
 * cover element and writes, host, out_d2[i*nrows + j] = the FP32 tile squared
 * distance n_i + n_j - 2 g_ij rescaled to the cloud's units, and
 * out_band[i*nrows+j] = the half-width of the certified band around it. */
mapper_status mapper_debug_tile_d2(mapper_context *ctx, const mapper_cloud *cloud,
                                   const int32_t *rows, int32_t nrows, int32_t precision,
                                   double eps, double *out_d2, double *out_band);

/* mapper_knn_d2 for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same k-th nearest-neighbour squared distances, bit for bit, with every
 * device work array (panels, bounds, candidate lists, counters) in a static
 * 64 MiB device array of the library, one per GPU, resolved when the first
 * context on that GPU is created; no hipMalloc, hipFree or arena use, and no
 * host allocation.
 *   points  device, n x d FP32 row-major (caller-owned, read only);
 *   out_d2  device, n doubles (caller-owned): the k-th smallest canonical
 *           squared distance from each point to the others;
 *   k in [1, min(16, n - 1)]; precision as mapper_knn_d2 (AUTO = FP16).
 * Runs on the context's stream and returns when the result is written.
 * Returns MAPPER_EINVAL, before any launch, when the work arrays of n x d
 * exceed the 64 MiB (about n = 30,000 at d = 256; the message states the
 * bytes needed), and when many equal distances make the candidate lists
 * outgrow it.  Calls on one GPU share its array: the library serializes them
 * (a lock held for the call), so two calls on one GPU never overlap; work of
 * other entry points is not affected.  The array keeps the last call's
 * contents; every piece a call relies on is cleared or rewritten first. */
mapper_status mapper_knn_d2_noalloc(mapper_context *ctx, const float *points, int64_t n, int32_t d, int32_t k,
                                    int32_t precision, double *out_d2);

/* Lens values of one axis (the first stage of mapper_run, same kernels;
 * n_intervals, overlap and cover are ignored): out (host, n doubles) gets the
 * canonical FP64 lens of every point (Background section: the filter
 * function).  Checks the lens, including the correctly rounded square root
 * of the L2 filter, against the oracle at any size. */
mapper_status mapper_debug_lens(mapper_context *ctx, const mapper_cloud *cloud, const mapper_axis *axis,
                                double *out);

/* The library's FP64 square root (the kernel that finishes the whole-cloud
 * lenses) on n host doubles: out[i] = sqrt(in[i]), to be checked against the
 * correctly rounded IEEE square root.  in and out are host memory. */
mapper_status mapper_debug_sqrt(mapper_context *ctx, const double *in, int64_t n, double *out);

#ifdef __cplusplus
}
#endif
#endif /* MAPPER_GPU_H */
