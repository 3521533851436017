// cells.hip -- a locality order for the members of each cover element, and
// the screening of distance tiles that cannot hold a neighbour pair.
//
// DBSCAN (Ester et al.) inside a pullback set needs the pairs within eps of
// each other; the paper's all-pairs query (Scalability section) computes all
// of them.  Most pairs of a large element are far apart when the cloud has
// cluster structure, so the library lays each element's members out in the
// order of a coarse partition of the cloud (its "cells": the nearest of up
// to 64 landmarks chosen by farthest-point sampling), and bounds every
// 128-row tile by a ball (its mean and the largest distance of a member from
// it).  A tile pair whose balls lie more than eps apart holds no neighbour
// pair (triangle inequality) and is not computed; so is a tile pair none of
// whose cells are near each other (each cell bounded by its own ball, the
// landmark and the largest distance of a member from it).  The partition
// only orders the work; the graph does not depend on it.
#include "internal.h"

namespace mgpu {

namespace {

constexpr int CB = 256;       // points per block (one per thread)
constexpr int CC = 32;        // columns per LDS slab

// cell[i] = the landmark nearest to point i (smallest |l|^2 - 2 x.l, FP32;
// the order is a heuristic, so rounding does not matter), or the outlier
// cell ncell when the point lies farther from it than limit2 (squared).
// Landmarks are staged whole in LDS (ncell * d <= CELL_LDS_FLOATS).
__global__ void __launch_bounds__(CB) k_assign_cells(const float *__restrict__ X, int64_t n, int32_t d,
                                                     const float *__restrict__ land, int32_t ncell,
                                                     const float *__restrict__ limit2, uint8_t *__restrict__ cell) {
    __shared__ float L[CELL_LDS_FLOATS];
    __shared__ float tile[CB][CC + 1];
    __shared__ float lnorm[CELL_MAX];
    for (int i = threadIdx.x; i < ncell * d; i += CB) L[i] = land[i];
    __syncthreads();
    if (threadIdx.x < ncell) {
        float s = 0.f;
        for (int j = 0; j < d; ++j) s += L[threadIdx.x * d + j] * L[threadIdx.x * d + j];
        lnorm[threadIdx.x] = s;
    }
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
            nx += x * x;
#pragma unroll
            for (int c = 0; c < CELL_MAX; ++c)
                if (c < ncell) acc[c] += x * L[c * d + c0 + j];
        }
    }
    const int64_t my = row0 + threadIdx.x;
    if (my >= n) return;
    int best = 0;
    float bv = lnorm[0] - 2.f * acc[0];
#pragma unroll
    for (int c = 1; c < CELL_MAX; ++c)
        if (c < ncell) {
            const float v = lnorm[c] - 2.f * acc[c];
            if (v < bv) { bv = v; best = c; }
        }
    // |x|^2 + bv is the squared distance to the landmark: beyond the cell's
    // limit the point goes to the outlier cell (id ncell)
    cell[my] = (uint8_t)(nx + bv > limit2[best] ? ncell : best);
}

// out[i] = min over j != i of |x_i - x_j|^2 among the m sample rows (FP32;
// it only separates isolated rows from rows in dense regions).
__global__ void k_sample_nn2(const float *__restrict__ sub, int32_t m, int32_t d, float *__restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const float *x = sub + (int64_t)i * d;
    float best = 3.0e38f;
    for (int j = 0; j < m; ++j) {
        if (j == i) continue;
        const float *y = sub + (int64_t)j * d;
        float acc = 0.f;
        for (int k = 0; k < d; ++k) {
            const float t = x[k] - y[k];
            acc += t * t;
        }
        best = acc < best ? acc : best;
    }
    out[i] = best;
}

// r2[c] = max over the points of cell c of |x - l_c|^2 (FP64 sums of
// squares of FP32 differences), as the bits of a non-negative double, which
// order like the values.
__global__ void k_cell_radius(const float *__restrict__ X, int64_t n, int32_t d, const float *__restrict__ land,
                              int32_t ncell, const uint8_t *__restrict__ cell, unsigned long long *__restrict__ r2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int c = cell[i];
    if (c >= ncell) return;                          // the outlier cell has no ball
    const float *x = X + i * (int64_t)d, *l = land + (int64_t)c * d;
    double acc = 0.0;
    for (int j = 0; j < d; ++j) {
        const double t = (double)x[j] - (double)l[j];
        acc += t * t;
    }
    atomicMax(&r2[c], (unsigned long long)__double_as_longlong(acc));
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

// Ball of each 128-slot row block: center c = the rows' mean, rounded to
// FP32; radius r >= max over the rows of |x - c| (FP64 sums of exact
// squares of FP32 differences, square root, then a relative margin of
// 2^-40, which covers the roundings for d <= BALL_DMAX).  One workgroup
// (four waves) per row block.
__global__ void __launch_bounds__(256) k_tile_balls(const float *__restrict__ X, int32_t d,
                                                    const uint32_t *__restrict__ slot_point,
                                                    const int64_t *__restrict__ elem_off,
                                                    const int64_t *__restrict__ rb_off, int32_t n_elem,
                                                    const uint8_t *__restrict__ cell,
                                                    const unsigned long long *__restrict__ near,
                                                    float *__restrict__ centers, double *__restrict__ radius,
                                                    unsigned long long *__restrict__ cmask,
                                                    unsigned long long *__restrict__ nmask) {
    __shared__ double part[4];
    __shared__ unsigned long long cm[4], nm[4];
    __shared__ float c[BALL_DMAX];
    const int64_t rb = blockIdx.x;
    const int e = rb_element(rb_off, n_elem, rb);
    const int64_t I = rb - rb_off[e];
    const int64_t s0 = elem_off[e] + I * TILE;
    const int64_t s1 = min(elem_off[e + 1], s0 + (int64_t)TILE);
    const int rows = (int)(s1 - s0);
    for (int j = threadIdx.x; j < d; j += blockDim.x) {
        double acc = 0.0;
        for (int r = 0; r < rows; ++r) acc += (double)X[(int64_t)slot_point[s0 + r] * d + j];
        c[j] = (float)(acc / rows);
        centers[rb * (int64_t)d + j] = c[j];
    }
    __syncthreads();
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    // the cells present among the rows, and the cells near any of them
    unsigned long long mc = 0, mn = 0;
    for (int r = threadIdx.x; r < rows; r += blockDim.x) {
        const int c = cell[slot_point[s0 + r]];
        mc |= 1ull << c;
        mn |= near[c];
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) {
        mc |= __shfl_xor(mc, o, WAVE);
        mn |= __shfl_xor(mn, o, WAVE);
    }
    if (lane == 0) {
        cm[w] = mc;
        nm[w] = mn;
    }
    double worst = 0.0;
    for (int r = w; r < rows; r += 4) {
        const float *x = X + (int64_t)slot_point[s0 + r] * d;
        double acc = 0.0;
        for (int j = lane; j < d; j += WAVE) {
            const double t = (double)x[j] - (double)c[j];
            acc += t * t;
        }
        for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
        worst = acc > worst ? acc : worst;
    }
    if (lane == 0) part[w] = worst;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(part[0], part[1]), fmax(part[2], part[3]));
        radius[rb] = sqrt(m) * (1.0 + 0x1.0p-40);
        cmask[rb] = cm[0] | cm[1] | cm[2] | cm[3];
        nmask[rb] = nm[0] | nm[1] | nm[2] | nm[3];
    }
}

// keep[i] = 0 when tile pair i provably holds no pair within eps: with the
// balls (c_I, r_I), (c_J, r_J), every x in I and y in J satisfy
// |x - y| >= |c_I - c_J| - r_I - r_J (triangle inequality), and the
// canonical FP64 distance is at least (1 - (d + 1) 2^-53) |x - y|^2.  The
// center distance is summed in FP64 from exact squares of FP32 differences
// and shrunk by 2^-40; the test keeps a further relative margin.  One wave
// per tile pair.
__global__ void __launch_bounds__(256) k_screen(const TileItem *__restrict__ items, int64_t n,
                                                const int64_t *__restrict__ rb_off, const float *__restrict__ centers,
                                                const double *__restrict__ radius,
                                                const unsigned long long *__restrict__ cmask,
                                                const unsigned long long *__restrict__ nmask, int32_t d, double E,
                                                uint8_t *__restrict__ keep) {
    const int64_t i = block_linear() * 4 + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (i >= n) return;
    const TileItem it = items[i];
    if (it.I == it.J) {
        if (lane == 0) keep[i] = 1;
        return;
    }
    const int64_t a = rb_off[it.e] + it.I, b = rb_off[it.e] + it.J;
    // no cell of tile J is near a cell of tile I: every pair is farther
    // than eps (the cells' own balls prove it)
    if ((nmask[a] & cmask[b]) == 0) {
        if (lane == 0) keep[i] = 0;
        return;
    }
    const float *ca = centers + a * (int64_t)d, *cb = centers + b * (int64_t)d;
    double acc = 0.0;
    for (int j = lane; j < d; j += WAVE) {
        const double t = (double)ca[j] - (double)cb[j];
        acc += t * t;
    }
    for (int o = WAVE / 2; o > 0; o >>= 1) acc += __shfl_xor(acc, o, WAVE);
    if (lane != 0) return;
    const double gap = sqrt(acc) * (1.0 - 0x1.0p-40) - radius[a] - radius[b];
    const double shrink = 1.0 - ((double)d + 8.0) * 0x1.0p-52;
    keep[i] = (gap > 0.0 && gap * gap * shrink > E * (1.0 + 0x1.0p-40)) ? 0 : 1;
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
    // every lane of the wave reaches here
    for (int o = WAVE / 2; o > 0; o >>= 1) np += __shfl_xor(np, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0 && np) atomicAdd(pairs, np);
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

hipError_t launch_tile_balls(const float *X, int32_t d, const uint32_t *slot_point, const int64_t *elem_off,
                             const int64_t *rb_off, int32_t n_elem, int64_t nrb, const uint8_t *cell,
                             const unsigned long long *near, float *centers, double *radius,
                             unsigned long long *cmask, unsigned long long *nmask, hipStream_t s) {
    if (nrb <= 0) return hipSuccess;
    if (nrb > 0x7fffffff || d > BALL_DMAX) return hipErrorInvalidValue;
    k_tile_balls<<<dim3((unsigned)nrb), dim3(256), 0, s>>>(X, d, slot_point, elem_off, rb_off, n_elem, cell, near,
                                                            centers, radius, cmask, nmask);
    return hipGetLastError();
}

hipError_t launch_screen(const TileItem *items, int64_t n, const int64_t *rb_off, const float *centers,
                         const double *radius, const unsigned long long *cmask, const unsigned long long *nmask,
                         int32_t d, double E, uint8_t *keep, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (d > BALL_DMAX) return hipErrorInvalidValue;
    k_screen<<<grid_2d((n + 3) / 4), dim3(256), 0, s>>>(items, n, rb_off, centers, radius, cmask, nmask, d, E,
                                                         keep);
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

hipError_t launch_assign_cells(const float *X, int64_t n, int32_t d, const float *land, int32_t ncell,
                               const float *limit2, uint8_t *cell, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (ncell < 1 || ncell >= CELL_MAX || (int64_t)ncell * d > CELL_LDS_FLOATS) return hipErrorInvalidValue;
    k_assign_cells<<<dim3((unsigned)((n + CB - 1) / CB)), dim3(CB), 0, s>>>(X, n, d, land, ncell, limit2, cell);
    return hipGetLastError();
}

hipError_t launch_sample_nn2(const float *sub, int32_t m, int32_t d, float *out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    k_sample_nn2<<<dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s>>>(sub, m, d, out);
    return hipGetLastError();
}

hipError_t launch_cell_radius(const float *X, int64_t n, int32_t d, const float *land, int32_t ncell,
                              const uint8_t *cell, unsigned long long *r2, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_cell_radius<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(X, n, d, land, ncell, cell, r2);
    return hipGetLastError();
}

hipError_t launch_shift_keys(uint64_t *keys, int64_t n, int shift, hipStream_t s) {
    if (n <= 0 || shift == 0) return hipSuccess;
    k_shift_keys<<<grid_2d((n + 255) / 256), dim3(256), 0, s>>>(keys, n, shift);
    return hipGetLastError();
}

}  // namespace mgpu
