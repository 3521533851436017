/*
 * mapper_oracle.c -- a plain, slow, FP64 CPU mapper.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code, header or constant with the GPU path.
 *
 * What it computes (Zhou et al., "Mapper Interactive", Background section):
 *   - a filter (lens) f : X -> R (1-D mapper) or R^2 (2-D mapper);
 *   - a cover V = {V_k} of f(X) by n intervals of equal length whose
 *     neighbours overlap by a fraction p (the paper's two cover parameters:
 *     the number of elements and their overlap, given as a percentage); for
 *     2-D the cover elements are the products of the two axes' intervals
 *     (rectangles);
 *   - for every cover element, DBSCAN (Ester et al.) of its pullback
 *     f^{-1}(V_k) with the Euclidean metric and parameters eps, minPts;
 *   - the mapper graph = 1-D nerve of the resulting clusters: one node per
 *     cluster, an edge between two nodes whose point sets intersect.
 *
 * Readings of points the paper leaves open (each one is a choice, listed in
 * the design notes with its justification):
 *   lens     column: (double)x_c;  L-inf: max_j |x_j|;
 *            L2: sqrt(S) with S = sum_j x_j*x_j accumulated in j order in FP64
 *            (each product of two floats is exact in FP64) and a correctly
 *            rounded sqrt;  projection on a float vector v: sum_j x_j*v_j in
 *            j order in FP64;  values: given;  k-NN distance (a density
 *            lens): sqrt of the k-th smallest D(x, y) over the other points,
 *            k = the axis' column field;  eccentricity (L-inf): sqrt of the
 *            largest D(x, y) over the other points.
 *   cover    L = (M-m)/(n-(n-1)p), s = L(1-p), lo_k = m + k s,
 *            hi_k = lo_k + L (k < n-1), hi_{n-1} = M; closed intervals.
 *   balanced the same formula on the rank axis [0, N-1] of the sorted lens
 *            values v_0 <= ... <= v_{N-1}, rounded outward to ranks:
 *            lo_k = v[floor(rlo_k)], hi_k = v[ceil(rhi_k)] (the balanced
 *            cover whose intervals hold equal numbers of points).
 *   distance D(a,b): t_j = (double)x_aj - (double)x_bj, D = fma(t_j,t_j,D)
 *            in j order starting from 0; neighbours iff D <= fl(eps*eps)
 *            (closed eps-ball); a point is its own neighbour.
 *   DBSCAN   core iff #neighbours >= minPts; clusters = connected components
 *            of core points under the neighbour relation; a non-core point
 *            with at least one core neighbour joins the lowest-numbered
 *            adjacent cluster; otherwise it is noise and is dropped.
 *   labels   cluster ids within an element ordered by the smallest member
 *            index of each component's core points; nodes ordered by
 *            (element id, cluster id), element id = k1*n2 + k2 for 2-D;
 *            node members ascending; edges (a<b) lexicographic, weight =
 *            number of shared points.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no -ffast-math).
 * Contraction is off so every expression rounds exactly as written.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)

enum { ORC_LENS_COLUMN = 0, ORC_LENS_L2 = 1, ORC_LENS_LINF = 2,
       ORC_LENS_PROJECTION = 3, ORC_LENS_VALUES = 4,
       ORC_LENS_KNN_DISTANCE = 5, ORC_LENS_ECCENTRICITY = 6 };

typedef struct {
    int32_t kind;
    int32_t column;
    const float *direction;   /* d floats (PROJECTION) */
    const double *values;     /* n doubles (VALUES) */
    int32_t n_intervals;
    double overlap;
    int32_t cover;            /* 0: uniform intervals; 1: balanced */
} orc_axis;

typedef struct {
    int64_t n_nodes, n_edges, n_elements, n_slots;
    int32_t *node_element;    /* n_nodes */
    int64_t *node_offsets;    /* n_nodes + 1 */
    int32_t *node_members;    /* node_offsets[n_nodes] */
    int32_t *edges;           /* 2 * n_edges */
    int32_t *edge_weights;    /* n_edges */
    /* stage dumps */
    double *lens;             /* n * n_axes, axis-major: lens[a*n + i] */
    double *lo, *hi;          /* per axis, n_intervals each, concatenated */
    int64_t *elem_offsets;    /* n_elements + 1 */
    int32_t *elem_members;    /* n_slots, ascending within an element */
    int32_t *slot_count;      /* neighbour count of each slot (self included) */
    uint8_t *slot_core;       /* 1 if core */
    int32_t *slot_node;       /* node id, or -1 for noise */
} orc_graph;

int orc_knn_d2(const float *X, int64_t n, int32_t d, int32_t k, double *out);
int orc_ecc_d2(const float *X, int64_t n, int32_t d, double *out);
double orc_pair_d2(const float *x, const float *y, int32_t d);

/* ------------------------------------------------------------------ lens */

/* Background section: the filter function f.  Canonical FP64 evaluation. */
int orc_lens(const float *X, int64_t n, int32_t d, const orc_axis *ax, double *f)
{
    for (int64_t i = 0; i < n; ++i) {
        const float *x = X + i * (int64_t)d;
        double v = 0.0;
        switch (ax->kind) {
        case ORC_LENS_COLUMN:
            v = (double)x[ax->column];
            break;
        case ORC_LENS_LINF:
            v = 0.0;
            for (int32_t j = 0; j < d; ++j) {
                double a = fabs((double)x[j]);
                if (a > v) v = a;
            }
            break;
        case ORC_LENS_L2: {
            double s = 0.0;
            for (int32_t j = 0; j < d; ++j) {
                double xj = (double)x[j];
                s = s + xj * xj;
            }
            v = sqrt(s);
            break;
        }
        case ORC_LENS_PROJECTION: {
            double s = 0.0;
            for (int32_t j = 0; j < d; ++j)
                s = s + (double)x[j] * (double)ax->direction[j];
            v = s;
            break;
        }
        case ORC_LENS_VALUES:
            v = ax->values[i];
            break;
        default:
            return ORC_EINVAL;
        }
        f[i] = v;
    }
    return 0;
}

/* ----------------------------------------------------------------- cover */

/* Background section: n intervals of uniform length, consecutive ones sharing a
 * fraction p of their length, covering [m, M] exactly. */
void orc_cover(double m, double M, int32_t n, double p, double *lo, double *hi)
{
    double L = (M - m) / ((double)n - (double)(n - 1) * p);
    double s = L * (1.0 - p);
    for (int32_t k = 0; k < n; ++k) {
        lo[k] = m + (double)k * s;
        hi[k] = (k == n - 1) ? M : lo[k] + L;
    }
}

/* ---------------------------------------------------------------- DBSCAN */

/* Squared distances from member a to members b in [b0, b1): for each pair the
 * FP64 fma chain over coordinates j = 0..d-1, in order.  XT holds the
 * element's coordinates as doubles, coordinate-major (XT[j*nk + b]). */
static void row_d2(const double *XT, int64_t nk, int32_t d, int64_t a,
                   int64_t b0, int64_t b1, double *D)
{
    for (int64_t b = b0; b < b1; ++b) D[b - b0] = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        const double *col = XT + (int64_t)j * nk;
        const double xa = col[a];
        for (int64_t b = b0; b < b1; ++b) {
            double t = xa - col[b];
            D[b - b0] = fma(t, t, D[b - b0]);
        }
    }
}

#define ORC_BLK 1024

static int64_t uf_find(int64_t *P, int64_t x)
{
    while (P[x] != x) {
        P[x] = P[P[x]];
        x = P[x];
    }
    return x;
}

static void uf_union(int64_t *P, int64_t a, int64_t b)
{
    a = uf_find(P, a);
    b = uf_find(P, b);
    if (a == b) return;
    if (a < b) P[b] = a; else P[a] = b;   /* the root is the smallest index */
}

static int orc_cmp_double(const void *a, const void *b)
{
    const double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Background section: the balanced cover, whose intervals hold equal
 * numbers of points.  The uniform cover is laid on the rank axis [0, N-1] of
 * the sorted lens values, and each rank interval [rlo, rhi] becomes the
 * value interval [v[floor(rlo)], v[ceil(rhi)]] (outward, so it is never
 * empty and the endpoints stay monotone).  A zero endpoint is stored as +0. */
int orc_cover_balanced(const double *f, int64_t n, int32_t nint, double p, double *lo, double *hi)
{
    double *v = (double *)malloc(sizeof(double) * (size_t)n);
    if (!v) return ORC_ENOMEM;
    memcpy(v, f, sizeof(double) * (size_t)n);
    qsort(v, (size_t)n, sizeof(double), orc_cmp_double);
    orc_cover(0.0, (double)(n - 1), nint, p, lo, hi);
    for (int32_t k = 0; k < nint; ++k) {
        int64_t a = (int64_t)floor(lo[k]), b = (int64_t)ceil(hi[k]);
        if (a < 0) a = 0;
        if (b > n - 1) b = n - 1;
        lo[k] = v[a] + 0.0;
        hi[k] = v[b] + 0.0;
    }
    free(v);
    return 0;
}

/* DBSCAN of one cover element (members idx[0..nk) in ascending order).
 * Outputs per member: neighbour count (self included), core flag and local
 * cluster id (-1 = noise).  Returns the number of clusters, or < 0 on error. */
int64_t orc_dbscan(const float *X, int32_t d, const int32_t *idx, int64_t nk,
                   double eps, int32_t min_pts, int32_t *count, uint8_t *core,
                   int32_t *cid)
{
    if (nk <= 0) return 0;
    const double E = eps * eps;
    double *XT = (double *)malloc(sizeof(double) * (size_t)nk * (size_t)d);
    int64_t *P = (int64_t *)malloc(sizeof(int64_t) * (size_t)nk);
    if (!XT || !P) { free(XT); free(P); return ORC_ENOMEM; }
    for (int64_t b = 0; b < nk; ++b)
        for (int32_t j = 0; j < d; ++j)
            XT[(int64_t)j * nk + b] = (double)X[(int64_t)idx[b] * d + j];

    /* 1. neighbour counts and core flags */
    int fail = 0;
#pragma omp parallel
    {
        double *D = (double *)malloc(sizeof(double) * ORC_BLK);
        if (!D) {
#pragma omp atomic write
            fail = 1;
        }
#pragma omp for schedule(dynamic, 8)
        for (int64_t a = 0; a < nk; ++a) {
            if (!D) continue;
            int32_t c = 0;
            for (int64_t b0 = 0; b0 < nk; b0 += ORC_BLK) {
                int64_t b1 = b0 + ORC_BLK < nk ? b0 + ORC_BLK : nk;
                row_d2(XT, nk, d, a, b0, b1, D);
                for (int64_t b = b0; b < b1; ++b) c += (D[b - b0] <= E);
            }
            count[a] = c;
            core[a] = (uint8_t)(c >= min_pts);
        }
        free(D);
    }
    if (fail) { free(XT); free(P); return ORC_ENOMEM; }

    /* 2. connected components of core points (union-find, root = min index).
     * Rows are processed in blocks: neighbour flags of a block are computed in
     * parallel, then the unions are applied in order. */
    for (int64_t a = 0; a < nk; ++a) P[a] = a;
    const int64_t RB = 64;
    uint8_t *adj = (uint8_t *)malloc((size_t)RB * (size_t)nk);
    if (!adj) { free(XT); free(P); return ORC_ENOMEM; }
    for (int64_t r0 = 0; r0 < nk; r0 += RB) {
        int64_t r1 = r0 + RB < nk ? r0 + RB : nk;
#pragma omp parallel
        {
            double *D = (double *)malloc(sizeof(double) * ORC_BLK);
#pragma omp for schedule(dynamic, 1)
            for (int64_t a = r0; a < r1; ++a) {
                uint8_t *row = adj + (a - r0) * nk;
                memset(row, 0, (size_t)nk);
                if (!core[a] || !D) continue;
                for (int64_t b0 = a + 1; b0 < nk; b0 += ORC_BLK) {
                    int64_t b1 = b0 + ORC_BLK < nk ? b0 + ORC_BLK : nk;
                    row_d2(XT, nk, d, a, b0, b1, D);
                    for (int64_t b = b0; b < b1; ++b)
                        row[b] = (uint8_t)(core[b] && D[b - b0] <= E);
                }
            }
            free(D);
        }
        for (int64_t a = r0; a < r1; ++a) {
            const uint8_t *row = adj + (a - r0) * nk;
            for (int64_t b = a + 1; b < nk; ++b)
                if (row[b]) uf_union(P, a, b);
        }
    }
    free(adj);

    /* 3. canonical cluster ids: components in order of their smallest core index */
    int64_t nclusters = 0;
    for (int64_t a = 0; a < nk; ++a) {
        cid[a] = -1;
        if (core[a] && uf_find(P, a) == a) cid[a] = (int32_t)nclusters++;
    }
    for (int64_t a = 0; a < nk; ++a)
        if (core[a]) cid[a] = cid[uf_find(P, a)];

    /* 4. border points: the lowest cluster id among adjacent core points */
#pragma omp parallel
    {
        double *D = (double *)malloc(sizeof(double) * ORC_BLK);
#pragma omp for schedule(dynamic, 8)
        for (int64_t a = 0; a < nk; ++a) {
            if (core[a] || !D) continue;
            int32_t best = -1;
            for (int64_t b0 = 0; b0 < nk; b0 += ORC_BLK) {
                int64_t b1 = b0 + ORC_BLK < nk ? b0 + ORC_BLK : nk;
                row_d2(XT, nk, d, a, b0, b1, D);
                for (int64_t b = b0; b < b1; ++b)
                    if (core[b] && D[b - b0] <= E && (best < 0 || cid[b] < best))
                        best = cid[b];
            }
            cid[a] = best;
        }
        free(D);
    }
    free(XT);
    free(P);
    return nclusters;
}

/* ---------------------------------------------------------------- mapper */

static int cmp_pair(const void *x, const void *y)
{
    const int32_t *a = (const int32_t *)x, *b = (const int32_t *)y;
    if (a[0] != b[0]) return a[0] < b[0] ? -1 : 1;
    if (a[1] != b[1]) return a[1] < b[1] ? -1 : 1;
    return 0;
}

void orc_graph_free(orc_graph *g)
{
    if (!g) return;
    free(g->node_element); free(g->node_offsets); free(g->node_members);
    free(g->edges); free(g->edge_weights); free(g->lens); free(g->lo); free(g->hi);
    free(g->elem_offsets); free(g->elem_members); free(g->slot_count);
    free(g->slot_core); free(g->slot_node);
    free(g);
}

int orc_validate(const float *X, int64_t n, int32_t d, int32_t n_axes,
                 const orc_axis *axes, double eps, int32_t min_pts)
{
    if (!X || n < 1 || n > 2147483647LL || d < 1) return ORC_EINVAL;
    if (n_axes < 1 || n_axes > 2) return ORC_EINVAL;
    if (!(eps >= 0.0) || !isfinite(eps) || min_pts < 1) return ORC_EINVAL;
    for (int32_t a = 0; a < n_axes; ++a) {
        const orc_axis *ax = &axes[a];
        if (ax->n_intervals < 1) return ORC_EINVAL;
        if (!(ax->overlap >= 0.0 && ax->overlap < 1.0)) return ORC_EINVAL;
        if (ax->cover < 0 || ax->cover > 1) return ORC_EINVAL;
        if (ax->kind == ORC_LENS_COLUMN && (ax->column < 0 || ax->column >= d)) return ORC_EINVAL;
        if (ax->kind == ORC_LENS_PROJECTION) {
            if (!ax->direction) return ORC_EINVAL;
            for (int32_t j = 0; j < d; ++j) if (!isfinite(ax->direction[j])) return ORC_EINVAL;
        }
        if (ax->kind == ORC_LENS_VALUES) {
            if (!ax->values) return ORC_EINVAL;
            for (int64_t i = 0; i < n; ++i) if (!isfinite(ax->values[i])) return ORC_EINVAL;
        }
        if (ax->kind < 0 || ax->kind > 6) return ORC_EINVAL;
        if (ax->kind == ORC_LENS_KNN_DISTANCE && (ax->column < 1 || (int64_t)ax->column > n - 1)) return ORC_EINVAL;
        if (ax->kind == ORC_LENS_ECCENTRICITY && n < 2) return ORC_EINVAL;
    }
    for (int64_t i = 0; i < n * (int64_t)d; ++i) if (!isfinite(X[i])) return ORC_EINVAL;
    return 0;
}

int orc_mapper(const float *X, int64_t n, int32_t d, int32_t n_axes,
               const orc_axis *axes, double eps, int32_t min_pts, orc_graph **out)
{
    *out = NULL;
    int rc = orc_validate(X, n, d, n_axes, axes, eps, min_pts);
    if (rc) return rc;
    orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
    if (!g) return ORC_ENOMEM;

    /* lens, range, cover per axis */
    int32_t nint[2] = {1, 1};
    int64_t tot_int = 0;
    for (int32_t a = 0; a < n_axes; ++a) { nint[a] = axes[a].n_intervals; tot_int += nint[a]; }
    g->lens = (double *)malloc(sizeof(double) * (size_t)(n * n_axes));
    g->lo = (double *)malloc(sizeof(double) * (size_t)tot_int);
    g->hi = (double *)malloc(sizeof(double) * (size_t)tot_int);
    if (!g->lens || !g->lo || !g->hi) { orc_graph_free(g); return ORC_ENOMEM; }
    double *lo[2], *hi[2], *f[2];
    int64_t ioff = 0;
    for (int32_t a = 0; a < n_axes; ++a) {
        f[a] = g->lens + (int64_t)a * n;
        if (axes[a].kind == ORC_LENS_KNN_DISTANCE || axes[a].kind == ORC_LENS_ECCENTRICITY) {
            rc = axes[a].kind == ORC_LENS_KNN_DISTANCE ? orc_knn_d2(X, n, d, axes[a].column, f[a])
                                                       : orc_ecc_d2(X, n, d, f[a]);
            for (int64_t i = 0; i < n && !rc; ++i) f[a][i] = sqrt(f[a][i]);
        } else {
            rc = orc_lens(X, n, d, &axes[a], f[a]);
        }
        if (rc) { orc_graph_free(g); return rc; }
        double m = f[a][0], M = f[a][0];
        for (int64_t i = 1; i < n; ++i) {
            if (f[a][i] < m) m = f[a][i];
            if (f[a][i] > M) M = f[a][i];
        }
        lo[a] = g->lo + ioff;
        hi[a] = g->hi + ioff;
        if (axes[a].cover == 1) {
            rc = orc_cover_balanced(f[a], n, nint[a], axes[a].overlap, lo[a], hi[a]);
            if (rc) { orc_graph_free(g); return rc; }
        } else {
            orc_cover(m, M, nint[a], axes[a].overlap, lo[a], hi[a]);
        }
        for (int32_t k = 0; k < nint[a]; ++k)        /* a range too wide for FP64 endpoints */
            if (!isfinite(lo[a][k]) || !isfinite(hi[a][k])) { orc_graph_free(g); return ORC_EINVAL; }
        ioff += nint[a];
    }

    /* cover elements and their members (ascending point index) */
    const int64_t nelem = (int64_t)nint[0] * (n_axes == 2 ? nint[1] : 1);
    g->n_elements = nelem;
    g->elem_offsets = (int64_t *)calloc((size_t)nelem + 1, sizeof(int64_t));
    if (!g->elem_offsets) { orc_graph_free(g); return ORC_ENOMEM; }
    for (int pass = 0; pass < 2; ++pass) {
        int64_t pos = 0;
        for (int64_t e = 0; e < nelem; ++e) {
            int32_t k1 = (int32_t)(n_axes == 2 ? e / nint[1] : e);
            int32_t k2 = (int32_t)(n_axes == 2 ? e % nint[1] : 0);
            if (pass == 0) g->elem_offsets[e] = pos;
            for (int64_t i = 0; i < n; ++i) {
                int in = lo[0][k1] <= f[0][i] && f[0][i] <= hi[0][k1];
                if (n_axes == 2) in = in && lo[1][k2] <= f[1][i] && f[1][i] <= hi[1][k2];
                if (in) {
                    if (pass == 1) g->elem_members[pos] = (int32_t)i;
                    ++pos;
                }
            }
        }
        if (pass == 0) {
            g->elem_offsets[nelem] = pos;
            g->n_slots = pos;
            g->elem_members = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pos + 1));
            g->slot_count = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pos + 1));
            g->slot_core = (uint8_t *)malloc((size_t)(pos + 1));
            g->slot_node = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pos + 1));
            if (!g->elem_members || !g->slot_count || !g->slot_core || !g->slot_node) {
                orc_graph_free(g); return ORC_ENOMEM;
            }
        }
    }

    /* DBSCAN per element; node ids in (element, cluster) order */
    int64_t nnodes = 0;
    int64_t *elem_first_node = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nelem + 1));
    if (!elem_first_node) { orc_graph_free(g); return ORC_ENOMEM; }
    for (int64_t e = 0; e < nelem; ++e) {
        int64_t s0 = g->elem_offsets[e], s1 = g->elem_offsets[e + 1];
        elem_first_node[e] = nnodes;
        int64_t nc = orc_dbscan(X, d, g->elem_members + s0, s1 - s0, eps, min_pts,
                                g->slot_count + s0, g->slot_core + s0, g->slot_node + s0);
        if (nc < 0) { free(elem_first_node); orc_graph_free(g); return (int)nc; }
        for (int64_t s = s0; s < s1; ++s)
            if (g->slot_node[s] >= 0) g->slot_node[s] += (int32_t)nnodes;
        nnodes += nc;
    }
    elem_first_node[nelem] = nnodes;
    g->n_nodes = nnodes;

    /* node CSR: members of a node come from one element, already ascending */
    g->node_element = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnodes + 1));
    g->node_offsets = (int64_t *)calloc((size_t)nnodes + 1, sizeof(int64_t));
    int64_t nmem = 0;
    for (int64_t s = 0; s < g->n_slots; ++s) nmem += (g->slot_node[s] >= 0);
    g->node_members = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nmem + 1));
    if (!g->node_element || !g->node_offsets || !g->node_members) {
        free(elem_first_node); orc_graph_free(g); return ORC_ENOMEM;
    }
    for (int64_t e = 0; e < nelem; ++e)
        for (int64_t v = elem_first_node[e]; v < elem_first_node[e + 1]; ++v)
            g->node_element[v] = (int32_t)e;
    for (int64_t s = 0; s < g->n_slots; ++s)
        if (g->slot_node[s] >= 0) g->node_offsets[g->slot_node[s] + 1]++;
    for (int64_t v = 0; v < nnodes; ++v) g->node_offsets[v + 1] += g->node_offsets[v];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnodes + 1));
    if (!fill) { free(elem_first_node); orc_graph_free(g); return ORC_ENOMEM; }
    memcpy(fill, g->node_offsets, sizeof(int64_t) * (size_t)(nnodes + 1));
    for (int64_t s = 0; s < g->n_slots; ++s) {
        int32_t v = g->slot_node[s];
        if (v >= 0) g->node_members[fill[v]++] = g->elem_members[s];
    }
    free(fill);
    free(elem_first_node);

    /* edges: nodes sharing a point (nerve of the clusters) */
    int64_t *pt_cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!pt_cnt) { orc_graph_free(g); return ORC_ENOMEM; }
    for (int64_t k = 0; k < nmem; ++k) pt_cnt[g->node_members[k] + 1]++;
    for (int64_t i = 0; i < n; ++i) pt_cnt[i + 1] += pt_cnt[i];
    int32_t *pt_nodes = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nmem + 1));
    int64_t *pfill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!pt_nodes || !pfill) { free(pt_cnt); free(pt_nodes); free(pfill); orc_graph_free(g); return ORC_ENOMEM; }
    memcpy(pfill, pt_cnt, sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t v = 0; v < nnodes; ++v)          /* nodes in ascending order */
        for (int64_t k = g->node_offsets[v]; k < g->node_offsets[v + 1]; ++k)
            pt_nodes[pfill[g->node_members[k]]++] = (int32_t)v;
    free(pfill);
    int64_t npairs = 0;
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = pt_cnt[i + 1] - pt_cnt[i];
        npairs += c * (c - 1) / 2;
    }
    int32_t *pairs = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(npairs + 1));
    if (!pairs) { free(pt_cnt); free(pt_nodes); orc_graph_free(g); return ORC_ENOMEM; }
    int64_t q = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t x = pt_cnt[i]; x < pt_cnt[i + 1]; ++x)
            for (int64_t y = x + 1; y < pt_cnt[i + 1]; ++y) {
                pairs[2 * q] = pt_nodes[x];
                pairs[2 * q + 1] = pt_nodes[y];
                ++q;
            }
    free(pt_cnt);
    free(pt_nodes);
    qsort(pairs, (size_t)npairs, 2 * sizeof(int32_t), cmp_pair);
    int64_t ne = 0;
    for (int64_t k = 0; k < npairs; ++k)
        if (k == 0 || cmp_pair(pairs + 2 * k, pairs + 2 * (k - 1)) != 0) ++ne;
    g->n_edges = ne;
    g->edges = (int32_t *)malloc(sizeof(int32_t) * 2 * (size_t)(ne + 1));
    g->edge_weights = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ne + 1));
    if (!g->edges || !g->edge_weights) { free(pairs); orc_graph_free(g); return ORC_ENOMEM; }
    int64_t e = -1;
    for (int64_t k = 0; k < npairs; ++k) {
        if (k == 0 || cmp_pair(pairs + 2 * k, pairs + 2 * (k - 1)) != 0) {
            ++e;
            g->edges[2 * e] = pairs[2 * k];
            g->edges[2 * e + 1] = pairs[2 * k + 1];
            g->edge_weights[e] = 0;
        }
        g->edge_weights[e]++;
    }
    free(pairs);
    *out = g;
    return 0;
}

/* Squared distances of all ordered pairs of the given rows (m x m, row-major),
 * each by the canonical chain (the DBSCAN neighbour routine above), rows in
 * parallel.  For the band-soundness tests of the GPU tiles. */
int orc_all_d2(const float *X, int64_t n, int32_t d, const int32_t *rows, int64_t m, double *out)
{
    if (!X || !rows || !out || m < 0 || d < 1) return ORC_EINVAL;
    for (int64_t k = 0; k < m; ++k)
        if (rows[k] < 0 || rows[k] >= n) return ORC_EINVAL;
    double *XT = (double *)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1) * (size_t)d);
    if (!XT) return ORC_ENOMEM;
    for (int64_t k = 0; k < m; ++k)
        for (int32_t j = 0; j < d; ++j) XT[(int64_t)j * m + k] = (double)X[(int64_t)rows[k] * d + j];
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t a = 0; a < m; ++a) row_d2(XT, m, d, a, 0, m, out + a * m);
    free(XT);
    return 0;
}

/* k-th nearest-neighbour squared distances (the eps-selection module of the
 * CIFAR-10 use case plots the distribution of the distances to the k-th
 * nearest neighbour).  out[i] = the k-th smallest canonical D(x_i, x_j) over
 * the other points j != i, ties counted with multiplicity, 1 <= k <= n-1.
 * The k smallest values of a row are kept in a sorted array. */
int orc_knn_d2(const float *X, int64_t n, int32_t d, int32_t k, double *out)
{
    if (!X || !out || n < 2 || d < 1 || k < 1 || (int64_t)k > n - 1) return ORC_EINVAL;
    double *XT = (double *)malloc(sizeof(double) * (size_t)n * (size_t)d);
    if (!XT) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < d; ++j) XT[(int64_t)j * n + i] = (double)X[i * (int64_t)d + j];
    int fail = 0;
#pragma omp parallel
    {
        double *D = (double *)malloc(sizeof(double) * (size_t)n);
        double *best = (double *)malloc(sizeof(double) * (size_t)k);
        if (!D || !best) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t a = 0; a < n; ++a) {
                row_d2(XT, n, d, a, 0, n, D);
                for (int32_t q = 0; q < k; ++q) best[q] = INFINITY;
                for (int64_t b = 0; b < n; ++b) {
                    if (b == a || !(D[b] < best[k - 1])) continue;
                    int32_t q = k - 1;                  /* insertion into the sorted k smallest */
                    while (q > 0 && best[q - 1] > D[b]) { best[q] = best[q - 1]; --q; }
                    best[q] = D[b];
                }
                out[a] = best[k - 1];
            }
        }
        free(D);
        free(best);
    }
    free(XT);
    return fail ? ORC_ENOMEM : 0;
}

/* orc_knn_d2 for the listed rows only (rows[q] in [0, n)): out[q] = the
 * k-th smallest canonical D(x_rows[q], x_j) over j != rows[q]. */
int orc_knn_d2_rows(const float *X, int64_t n, int32_t d, int32_t k, const int32_t *rows, int64_t m,
                    double *out)
{
    if (!X || !rows || !out || n < 2 || d < 1 || k < 1 || (int64_t)k > n - 1 || m < 0) return ORC_EINVAL;
    for (int64_t q = 0; q < m; ++q)
        if (rows[q] < 0 || rows[q] >= n) return ORC_EINVAL;
    int fail = 0;
#pragma omp parallel
    {
        double *best = (double *)malloc(sizeof(double) * (size_t)k);
        if (!best) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 1)
            for (int64_t q = 0; q < m; ++q) {
                const int64_t a = rows[q];
                for (int32_t s = 0; s < k; ++s) best[s] = INFINITY;
                for (int64_t b = 0; b < n; ++b) {
                    if (b == a) continue;
                    const double D = orc_pair_d2(X + a * (int64_t)d, X + b * (int64_t)d, d);
                    if (!(D < best[k - 1])) continue;
                    int32_t s = k - 1;
                    while (s > 0 && best[s - 1] > D) { best[s] = best[s - 1]; --s; }
                    best[s] = D;
                }
                out[q] = best[k - 1];
            }
        }
        free(best);
    }
    return fail ? ORC_ENOMEM : 0;
}

/* The eccentricity lens (Background and Design sections list eccentricity
 * among the filter functions): the L-infinity eccentricity of a point is its
 * largest distance to the other points; out[i] = max over j != i of the
 * canonical D(x_i, x_j) (its square root is the lens). */
int orc_ecc_d2(const float *X, int64_t n, int32_t d, double *out)
{
    if (!X || !out || n < 2 || d < 1) return ORC_EINVAL;
    double *XT = (double *)malloc(sizeof(double) * (size_t)n * (size_t)d);
    if (!XT) return ORC_ENOMEM;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t j = 0; j < d; ++j) XT[(int64_t)j * n + i] = (double)X[i * (int64_t)d + j];
    int fail = 0;
#pragma omp parallel
    {
        double *D = (double *)malloc(sizeof(double) * (size_t)n);
        if (!D) {
#pragma omp atomic write
            fail = 1;
        } else {
#pragma omp for schedule(dynamic, 16)
            for (int64_t a = 0; a < n; ++a) {
                row_d2(XT, n, d, a, 0, n, D);
                double m = 0.0;
                for (int64_t b = 0; b < n; ++b)
                    if (b != a && D[b] > m) m = D[b];
                out[a] = m;
            }
        }
        free(D);
    }
    free(XT);
    return fail ? ORC_ENOMEM : 0;
}

/* Threads an OpenMP region of the oracle runs on (for reporting timings). */
int orc_threads(void)
{
    return omp_get_max_threads();
}

/* Squared distance of one pair by the canonical chain (for pins and for the
 * tolerance tests of the GPU tiles). */
double orc_pair_d2(const float *x, const float *y, int32_t d)
{
    double D = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        double t = (double)x[j] - (double)y[j];
        D = fma(t, t, D);
    }
    return D;
}
