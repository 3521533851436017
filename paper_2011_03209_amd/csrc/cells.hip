// cells.hip -- a locality order for the members of each cover element, and
// the screening of distance tiles that cannot hold a neighbour pair.
//
// DBSCAN (Ester et al.) inside a pullback set needs the pairs within eps of
// each other; the paper's all-pairs query (Scalability section) computes all
// of them.  Most pairs of a large element are far apart when the cloud has
// cluster structure, so the library lays each element's members out in the
// order of a coarse partition of the cloud (its "cells": the nearest of up
// to 62 landmarks chosen by farthest-point sampling, plus one cell for
// outlying points), and bounds every landmark cell by a ball (the landmark
// and the largest distance of a member from it).  A tile pair none of whose
// cells are near each other (balls more than eps apart) holds no neighbour
// pair (triangle inequality) and is not computed.  Bounding each 128-row
// tile by a ball of its own as well screened no more than 0.1% extra tile
// pairs on the mixtures measured (members of one cell are in point order
// within it, so the tiles of one cell overlap), and it cost two more reads
// of every row, so it is not done.  A point of the outlier cell gets its own
// bound on the distance to every landmark cell, and one farther than eps
// from all of them can only neighbour other outliers.  The partition only
// orders the work; the graph does not depend on it.
#include "internal.h"

namespace mgpu {

namespace {

constexpr int CB = 256;       // points per block (one per thread)
constexpr int CC = 32;        // columns per LDS slab

// cell[i] = the landmark nearest to point i (smallest |l|^2 - 2 x.l, FP32;
// the order is a heuristic, so rounding does not matter), or the outlier
// cell ncell when the point lies farther from it than limit2 (squared).
// The landmarks come transposed (coordinate j of landmark c at
// landT[j * CELL_MAX + c], zero past ncell), so every thread reads the same
// 64 values per coordinate: wave-uniform loads that the FMAs take as scalar
// operands.  One point per thread, its row staged through LDS in slabs.
__global__ void __launch_bounds__(CB) k_assign_cells(const float *__restrict__ X, int64_t n, int32_t d,
                                                     const float *__restrict__ landT,
                                                     const float *__restrict__ lnorm, int32_t ncell,
                                                     const float *__restrict__ limit2, uint8_t *__restrict__ cell,
                                                     uint8_t *__restrict__ far) {
    __shared__ float tile[CB][CC + 1];
    const int64_t row0 = (int64_t)blockIdx.x * CB;
    float acc[CELL_MAX], nx = 0.f;
#pragma unroll
    for (int c = 0; c < CELL_MAX; ++c) acc[c] = 0.f;
    for (int32_t c0 = 0; c0 < d; c0 += CC) {
        const int cw = (d - c0) < CC ? (d - c0) : CC;
        __syncthreads();
        for (int q = 0; q < CB * CC / CB; ++q) {           // coalesced: 32 floats of a row per 32 threads
            const int idx = q * CB + threadIdx.x;
            const int r = idx / CC, j = idx % CC;
            const int64_t gr = row0 + r;
            tile[r][j] = (gr < n && j < cw) ? X[gr * d + c0 + j] : 0.f;
        }
        __syncthreads();
        for (int j = 0; j < cw; ++j) {
            const float x = tile[threadIdx.x][j];
            const float *lt = landT + (int64_t)(c0 + j) * CELL_MAX;
            nx += x * x;
#pragma unroll
            for (int c = 0; c < CELL_MAX; ++c) acc[c] += x * lt[c];
        }
    }
    const int64_t my = row0 + threadIdx.x;
    if (my >= n) return;
    int best = 0, worst = 0;
    float bv = lnorm[0] - 2.f * acc[0], wv = bv;
#pragma unroll
    for (int c = 1; c < CELL_MAX; ++c)
        if (c < ncell) {
            const float v = lnorm[c] - 2.f * acc[c];
            if (v < bv) { bv = v; best = c; }
            if (v > wv) { wv = v; worst = c; }
        }
    if (far) far[my] = (uint8_t)worst;                      // the farthest landmark (a hint, not a bound)
    // |x|^2 + bv is the squared distance to the landmark: beyond the cell's
    // limit the point goes to the outlier cell (id ncell)
    cell[my] = (uint8_t)(nx + bv > limit2[best] ? ncell : best);
}

// out[i] = min over j != i of |x_i - x_j|^2 among the m sample rows (FP32;
// it only separates isolated rows from rows in dense regions).  One
// workgroup per row i, its row in LDS; each wave takes every fourth row j,
// the lanes striding its coordinates (coalesced), a shuffle sum per j.
__global__ void __launch_bounds__(256) k_sample_nn2(const float *__restrict__ sub, int32_t m, int32_t d,
                                                    float *__restrict__ out) {
    __shared__ float xi[CELL_LDS_FLOATS / 8];
    __shared__ float part[4];
    const int i = blockIdx.x;
    const float *x = sub + (int64_t)i * d;
    for (int k = threadIdx.x; k < d; k += blockDim.x) xi[k] = x[k];
    __syncthreads();
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    float best = 3.0e38f;
    for (int j = w; j < m; j += 4) {
        if (j == i) continue;
        const float *y = sub + (int64_t)j * d;
        float acc = 0.f;
        for (int k = lane; k < d; k += WAVE) {
            const float t = xi[k] - y[k];
            acc += t * t;
        }
        for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
        best = acc < best ? acc : best;
    }
    if (lane == 0) part[w] = best;
    __syncthreads();
    if (threadIdx.x == 0) out[i] = fminf(fminf(part[0], part[1]), fminf(part[2], part[3]));
}

// r2[c] = max over the points of cell c of |x - l_c|^2 (FP64 sums of
// squares of FP32 differences), as the bits of a non-negative double, which
// order like the values.  A wave takes one point at a time, its lanes along
// the row; the workgroup's maxima meet in LDS, so each workgroup of
// CR_POINTS points issues at most one global atomic per cell.
constexpr int CR_POINTS = 256;

__global__ void __launch_bounds__(256) k_cell_radius(const float *__restrict__ X, int64_t n, int32_t d,
                                                     const float *__restrict__ land, int32_t ncell,
                                                     const uint8_t *__restrict__ cell,
                                                     unsigned long long *__restrict__ r2) {
    __shared__ unsigned long long bmax[CELL_MAX];
    if (threadIdx.x < CELL_MAX) bmax[threadIdx.x] = 0;
    __syncthreads();
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const int64_t p0 = block_linear() * CR_POINTS;
    for (int q = w; q < CR_POINTS; q += (int)(blockDim.x / WAVE)) {
        const int64_t i = p0 + q;
        if (i >= n) break;                                   // uniform across the wave
        const int c = cell[i];
        if (c >= ncell) continue;                            // the outlier cell has no ball
        const float *x = X + i * (int64_t)d, *l = land + (int64_t)c * d;
        double acc = 0.0;
        for (int j = lane; j < d; j += WAVE) {
            const double t = (double)x[j] - (double)l[j];
            acc += t * t;
        }
        for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
        if (lane == 0) atomicMax(&bmax[c], (unsigned long long)__double_as_longlong(acc));
    }
    __syncthreads();
    if (threadIdx.x < ncell && bmax[threadIdx.x]) atomicMax(&r2[threadIdx.x], bmax[threadIdx.x]);
}

// gap[i] <= min over the landmark cells c of |x_i - l_c| - r_c for a point
// of the outlier cell (FP64 sums of exact squares of FP32 differences,
// square root shrunk by 2^-40, rounded down to FP32): every point of every
// landmark cell lies at least gap[i] from x_i (triangle inequality).  -1 for
// the other points.  One wave per point.
__global__ void __launch_bounds__(256) k_outlier_gap(const float *__restrict__ X, int64_t n, int32_t d,
                                                     const float *__restrict__ land, int32_t ncell,
                                                     const double *__restrict__ rad,
                                                     const uint8_t *__restrict__ cell, float *__restrict__ gap) {
    const int64_t i = block_linear() * 4 + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (i >= n) return;                                      // the whole wave leaves together
    if (cell[i] != ncell) {
        if (lane == 0) gap[i] = -1.0f;
        return;
    }
    const float *x = X + i * (int64_t)d;
    double best = 1e300;
    for (int c = 0; c < ncell; ++c) {
        const float *l = land + (int64_t)c * d;
        double acc = 0.0;
        for (int j = lane; j < d; j += WAVE) {
            const double t = (double)x[j] - (double)l[j];
            acc += t * t;
        }
        for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
        const double g = sqrt(acc) * (1.0 - 0x1.0p-40) - rad[c];
        best = g < best ? g : best;
    }
    if (lane == 0) {
        float f = (float)best;                               // round down
        if ((double)f > best) f = __uint_as_float(f > 0.0f ? __float_as_uint(f) - 1u
                                                 : f == 0.0f ? 0x80000001u : __float_as_uint(f) + 1u);
        gap[i] = f;
    }
}

// keys[s] >>= shift (the element id of each slot after the sort by
// (element, cell)).
__global__ void k_shift_keys(uint64_t *keys, int64_t n, int shift) {
    const int64_t i = block_linear() * blockDim.x + threadIdx.x;
    if (i < n) keys[i] >>= shift;
}

// The row block (element e, block I) of linear row-block index rb: rb_off
// numbers the row blocks element by element.
__device__ __forceinline__ int rb_element(const int64_t *rb_off, int32_t n_elem, int64_t rb) {
    int lo = 0, hi = n_elem;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rb_off[mid] <= rb) lo = mid; else hi = mid;
    }
    return lo;
}

// The cells of each 128-slot row block: cmask = the cells of its rows,
// nmask = the cells near any of them (near[c]: the cells whose balls lie
// within eps of cell c's ball, c included).  A point of the outlier cell
// whose gap to every landmark cell exceeds eps (the same bound as between
// two cells) counts as cell outlier + 1, which is near outliers only.  One
// wave per row block.
__global__ void __launch_bounds__(256) k_tile_cells(const uint32_t *__restrict__ slot_point,
                                                    const int64_t *__restrict__ elem_off,
                                                    const int64_t *__restrict__ rb_off, int32_t n_elem, int64_t nrb,
                                                    const uint8_t *__restrict__ cell,
                                                    const float *__restrict__ ogap, int32_t outlier,
                                                    double shrink, double Eb,
                                                    const unsigned long long *__restrict__ near,
                                                    unsigned long long *__restrict__ cmask,
                                                    unsigned long long *__restrict__ nmask) {
    const int64_t rb = block_linear() * 4 + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (rb >= nrb) return;                                    // the whole wave leaves together
    const int e = rb_element(rb_off, n_elem, rb);
    const int64_t s0 = elem_off[e] + (rb - rb_off[e]) * TILE;
    const int64_t s1 = min(elem_off[e + 1], s0 + (int64_t)TILE);
    unsigned long long mc = 0, mn = 0;
    for (int64_t r = s0 + lane; r < s1; r += WAVE) {
        const uint32_t p = slot_point[r];
        int c = cell[p];
        if (c == outlier && ogap) {                            // farther than eps from every landmark cell
            const double g = (double)ogap[p];
            if (g > 0.0 && g * g * shrink > Eb) c = outlier + 1;
        }
        mc |= 1ull << c;
        mn |= near[c];
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        mc |= __shfl_xor(mc, o, WAVE);
        mn |= __shfl_xor(mn, o, WAVE);
    }
    if (lane == 0) {
        cmask[rb] = mc;
        nmask[rb] = mn;
    }
}

// keep[i] = 0 when tile pair i provably holds no pair within eps: no cell
// of row block J is near a cell of row block I, so the cells' balls put
// every pair of the two blocks farther apart than eps.  Diagonal pairs are
// always kept.
__global__ void k_screen(const TileItem *__restrict__ items, int64_t n, const int64_t *__restrict__ rb_off,
                         const unsigned long long *__restrict__ cmask, const unsigned long long *__restrict__ nmask,
                         uint8_t *__restrict__ keep) {
    const int64_t i = block_linear() * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const TileItem it = items[i];
    const int64_t a = rb_off[it.e] + it.I, b = rb_off[it.e] + it.J;
    keep[i] = (it.I == it.J || (nmask[a] & cmask[b]) != 0) ? 1 : 0;
}

// The kept tile pairs, in their launch order, each with its own bitmask
// block (its position); diag_blk / next_blk[rb_off[e] + I] = the blocks of
// kept pairs (I, I) and (I, I + 1) of element e (for the hooking pass).
__global__ void k_compact_items(const TileItem *__restrict__ items, int64_t n, const uint8_t *__restrict__ keep,
                                const int64_t *__restrict__ pos, const int64_t *__restrict__ rb_off,
                                TileItem *__restrict__ out, int64_t *__restrict__ diag_blk,
                                int64_t *__restrict__ next_blk, unsigned long long *__restrict__ pairs) {
    const int64_t i = block_linear() * blockDim.x + threadIdx.x;
    unsigned long long np = 0;                 // in-element pairs of the kept tile pair
    if (i < n) {
        TileItem it = items[i];
        const int64_t p = pos[i];
        const bool k = keep[i] != 0;
        if (it.J == it.I) diag_blk[rb_off[it.e] + it.I] = p;          // diagonal pairs are always kept
        if (it.J == it.I + 1) next_blk[rb_off[it.e] + it.I] = k ? p : -1;
        if (k) {
            const int64_t ri = min((int64_t)TILE, (int64_t)it.ne - (int64_t)it.I * TILE);
            const int64_t rj = min((int64_t)TILE, (int64_t)it.ne - (int64_t)it.J * TILE);
            np = it.I == it.J ? (unsigned long long)(ri * (ri + 1) / 2) : (unsigned long long)(ri * rj);
            it.blk = p;
            out[p] = it;
        }
    }
    // every thread of the workgroup reaches here: the workgroup's sum, one
    // atomic on one of PAIR_SLOTS counters (the caller adds them up), so
    // the launch does not queue on a single address
    for (int o = WAVE / 2; o > 0; o >>= 1) np += __shfl_xor(np, o, WAVE);
    __shared__ unsigned long long part[4];
    if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = np;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(&pairs[block_linear() % PAIR_SLOTS], t);
    }
}

__global__ void k_sample_items(const TileItem *__restrict__ items, int64_t n, int64_t m, TileItem *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    TileItem it = items[i * n / m];                  // i < m <= 8192: no overflow
    it.blk = i;
    out[i] = it;
}

}  // namespace

hipError_t launch_sample_items(const TileItem *items, int64_t n, int64_t m, TileItem *out, hipStream_t s) {
    if (m <= 0 || n <= 0 || m > n) return m <= 0 ? hipSuccess : hipErrorInvalidValue;
    k_sample_items<<<dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s>>>(items, n, m, out);
    return hipGetLastError();
}

hipError_t launch_tile_cells(const uint32_t *slot_point, const int64_t *elem_off, const int64_t *rb_off,
                             int32_t n_elem, int64_t nrb, const uint8_t *cell, const float *ogap, int32_t outlier,
                             double shrink, double Eb, const unsigned long long *near, unsigned long long *cmask,
                             unsigned long long *nmask, hipStream_t s) {
    if (nrb <= 0) return hipSuccess;
    if (outlier < 0 || outlier + 1 >= CELL_MAX) return hipErrorInvalidValue;
    k_tile_cells<<<grid_2d((nrb + 3) / 4), dim3(256), 0, s>>>(slot_point, elem_off, rb_off, n_elem, nrb, cell, ogap,
                                                               outlier, shrink, Eb, near, cmask, nmask);
    return hipGetLastError();
}

hipError_t launch_outlier_gap(const float *X, int64_t n, int32_t d, const float *land, int32_t ncell,
                              const double *rad, const uint8_t *cell, float *gap, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (ncell < 1 || ncell >= CELL_MAX) return hipErrorInvalidValue;
    k_outlier_gap<<<grid_2d((n + 3) / 4), dim3(256), 0, s>>>(X, n, d, land, ncell, rad, cell, gap);
    return hipGetLastError();
}

hipError_t launch_screen(const TileItem *items, int64_t n, const int64_t *rb_off, const unsigned long long *cmask,
                         const unsigned long long *nmask, uint8_t *keep, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_screen<<<grid_2d((n + 255) / 256), dim3(256), 0, s>>>(items, n, rb_off, cmask, nmask, keep);
    return hipGetLastError();
}

hipError_t launch_compact_items(const TileItem *items, int64_t n, const uint8_t *keep, const int64_t *pos,
                                const int64_t *rb_off, TileItem *out, int64_t *diag_blk, int64_t *next_blk,
                                unsigned long long *pairs, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_compact_items<<<grid_2d((n + 255) / 256), dim3(256), 0, s>>>(items, n, keep, pos, rb_off, out, diag_blk,
                                                                    next_blk, pairs);
    return hipGetLastError();
}

hipError_t launch_assign_cells(const float *X, int64_t n, int32_t d, const float *landT, const float *lnorm,
                               int32_t ncell, const float *limit2, uint8_t *cell, uint8_t *far, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (ncell < 1 || ncell + 1 >= CELL_MAX) return hipErrorInvalidValue;
    k_assign_cells<<<dim3((unsigned)((n + CB - 1) / CB)), dim3(CB), 0, s>>>(X, n, d, landT, lnorm, ncell, limit2,
                                                                          cell, far);
    return hipGetLastError();
}

hipError_t launch_sample_nn2(const float *sub, int32_t m, int32_t d, float *out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    if (d > CELL_LDS_FLOATS / 8) return hipErrorInvalidValue;
    k_sample_nn2<<<dim3((unsigned)m), dim3(256), 0, s>>>(sub, m, d, out);
    return hipGetLastError();
}

hipError_t launch_cell_radius(const float *X, int64_t n, int32_t d, const float *land, int32_t ncell,
                              const uint8_t *cell, unsigned long long *r2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (ncell < 1 || ncell >= CELL_MAX) return hipErrorInvalidValue;
    k_cell_radius<<<grid_2d((n + CR_POINTS - 1) / CR_POINTS), dim3(256), 0, s>>>(X, n, d, land, ncell, cell, r2);
    return hipGetLastError();
}

hipError_t launch_shift_keys(uint64_t *keys, int64_t n, int shift, hipStream_t s) {
    if (n <= 0 || shift == 0) return hipSuccess;
    k_shift_keys<<<grid_2d((n + 255) / 256), dim3(256), 0, s>>>(keys, n, shift);
    return hipGetLastError();
}

}  // namespace mgpu
