// lens.hip -- cloud validation, canonical FP64 lens values, lens range.
//
// Filter functions of the Background section (column, L2 norm, L-infinity
// norm, projection, given values).  The lens is evaluated once per point in
// FP64 with the coordinates taken in index order, so it is the same value on
// every device and in every run; interval membership is then an exact
// comparison.  The kernel is bound by HBM: it reads the n x d cloud once,
// staging 32-column slabs of 256 rows through LDS so that global loads are
// coalesced while each thread still walks its own row in order.
#include "internal.h"

namespace mgpu {

namespace {

constexpr int LB = 256;       // rows per block (one per thread)
constexpr int LC = 32;        // columns per LDS slab

__global__ void __launch_bounds__(256) k_check_cloud(const float *X, int64_t count, uint32_t *out) {
    // out[0]: 1 if a non-finite value was seen; out[1]: max |x| as float bits
    uint32_t bad = 0, mx = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t b = __float_as_uint(X[i]) & 0x7fffffffu;
        if (b >= 0x7f800000u) bad = 1; else mx = b > mx ? b : mx;
    }
    for (int o = 32; o > 0; o >>= 1) {
        bad |= __shfl_xor(bad, o, WAVE);
        const uint32_t t = __shfl_xor(mx, o, WAVE);
        mx = t > mx ? t : mx;
    }
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        if (bad) atomicOr(&out[0], 1u);
        atomicMax(&out[1], mx);
    }
}

__global__ void __launch_bounds__(LB) k_lens_rows(const float *__restrict__ X, int64_t n, int32_t d,
                                                  int kind, const float *__restrict__ dir,
                                                  double *__restrict__ f) {
    __shared__ float tile[LB][LC + 1];
    __shared__ double vdir[LC];
    const int64_t row0 = (int64_t)blockIdx.x * LB;
    const int64_t my = row0 + threadIdx.x;
    double acc = 0.0;
    // full slabs of rows with 16-byte alignment: 8 threads cover a slab's 128
    // bytes of a row, and the next slab's loads are issued before this one's
    // sums (they land while the chains run)
    constexpr int NQ = LB * LC / 4 / 256;
    const bool vec = (d & 3) == 0;
    float4 pre[NQ];
    auto load_slab = [&](int32_t c0) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const int idx = q * 256 + threadIdx.x;
            const int r = idx / (LC / 4), j = 4 * (idx % (LC / 4));
            const int64_t gr = row0 + r;
            pre[q] = gr < n ? *(const float4 *)(X + gr * d + c0 + j) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    };
    if (vec && d >= LC) load_slab(0);
    for (int32_t c0 = 0; c0 < d; c0 += LC) {
        const int cw = (d - c0) < LC ? (d - c0) : LC;
        if (vec && cw == LC) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) {
                const int idx = q * 256 + threadIdx.x;
                const int r = idx / (LC / 4), j = 4 * (idx % (LC / 4));
                tile[r][j] = pre[q].x;
                tile[r][j + 1] = pre[q].y;
                tile[r][j + 2] = pre[q].z;
                tile[r][j + 3] = pre[q].w;
            }
            if (c0 + 2 * LC <= d) load_slab(c0 + LC);
        } else {
            // coalesced load: 32 consecutive floats of a row per 32 threads
#pragma unroll 4
            for (int q = 0; q < LB * LC / 256; ++q) {
                const int idx = q * 256 + threadIdx.x;
                const int r = idx / LC, j = idx % LC;
                const int64_t gr = row0 + r;
                float v = 0.f;
                if (gr < n && j < cw) v = X[gr * d + c0 + j];
                tile[r][j] = v;
            }
        }
        if (kind == 3 && threadIdx.x < LC) vdir[threadIdx.x] = threadIdx.x < cw ? (double)dir[c0 + threadIdx.x] : 0.0;
        __syncthreads();
        if (my < n) {
            if (kind == 1) {            // L2: sum of exact squares, in order (the fma adds the exact square)
#pragma unroll 4
                for (int j = 0; j < cw; ++j) {
                    const double x = (double)tile[threadIdx.x][j];
                    acc = __builtin_fma(x, x, acc);
                }
            } else if (kind == 3) {     // projection: sum of exact products, in order
#pragma unroll 4
                for (int j = 0; j < cw; ++j) {
                    const double x = (double)tile[threadIdx.x][j];
                    acc = __builtin_fma(x, vdir[j], acc);
                }
            } else {                    // L-infinity
#pragma unroll 4
                for (int j = 0; j < cw; ++j) {
                    const double x = fabs((double)tile[threadIdx.x][j]);
                    acc = x > acc ? x : acc;
                }
            }
        }
        __syncthreads();
    }
    if (my < n) f[my] = (kind == 1) ? sqrt(acc) : acc;
}

__global__ void k_lens_column(const float *X, int64_t n, int32_t d, int32_t c, double *f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] = (double)X[i * d + c];
}

__global__ void k_lens_values(const double *v, int64_t n, double *f) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] = v[i];
}

// Order-preserving map of doubles to unsigned keys (no NaNs reach here).
__device__ __forceinline__ unsigned long long dkey(double x) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(x);
    return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// One atomic pair per workgroup (the waves' results meet in LDS first): the
// two words are shared by the whole launch.
__global__ void __launch_bounds__(256) k_range(const double *f, int64_t n, unsigned long long *keys2) {
    __shared__ unsigned long long wmn[4], wmx[4];
    unsigned long long mn = ~0ull, mx = 0ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long k = dkey(f[i]);
        mn = k < mn ? k : mn;
        mx = k > mx ? k : mx;
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long a = __shfl_xor(mn, o, WAVE);
        const unsigned long long b = __shfl_xor(mx, o, WAVE);
        mn = a < mn ? a : mn;
        mx = b > mx ? b : mx;
    }
    const int w = threadIdx.x / WAVE;
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        wmn[w] = mn;
        wmx[w] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int v = 1; v < (int)(blockDim.x / WAVE); ++v) {
            mn = wmn[v] < mn ? wmn[v] : mn;
            mx = wmx[v] > mx ? wmx[v] : mx;
        }
        atomicMin(&keys2[0], mn);
        atomicMax(&keys2[1], mx);
    }
}

// Balanced cover (the cover whose intervals hold equal numbers of points,
// Background section): the lens as ordered keys for a radix sort ...
__global__ void k_lens_keys(const double *f, int64_t n, uint64_t *keys, uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    keys[i] = dkey(f[i]);
    vals[i] = (uint32_t)i;
}

// ... and the lens values of given ranks read back from the sorted keys (a
// zero comes back as +0).
__global__ void k_rank_values(const uint64_t *sorted, const int64_t *rank, int32_t m, double *out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const unsigned long long k = sorted[rank[i]];
    const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
    out[i] = __longlong_as_double((long long)b) + 0.0;
}

__global__ void k_sqrt(double *f, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) f[i] = sqrt(f[i]);
}

}  // namespace

hipError_t launch_sqrt(double *f, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_sqrt<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(f, n);
    return hipGetLastError();
}

hipError_t launch_lens_keys(const double *f, int64_t n, uint64_t *keys, uint32_t *vals, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_lens_keys<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(f, n, keys, vals);
    return hipGetLastError();
}

hipError_t launch_rank_values(const uint64_t *sorted, const int64_t *rank, int32_t m, double *out,
                              hipStream_t s) {
    if (m <= 0) return hipSuccess;
    k_rank_values<<<dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s>>>(sorted, rank, m, out);
    return hipGetLastError();
}

hipError_t launch_check_cloud(const float *X, int64_t count, uint32_t *flags_maxabs, hipStream_t s) {
    int64_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (blocks < 1) blocks = 1;
    k_check_cloud<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(X, count, flags_maxabs);
    return hipGetLastError();
}

hipError_t launch_lens(const float *X, int64_t n, int32_t d, int kind, int32_t column,
                       const float *dir, const double *values, double *f, hipStream_t s) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    switch (kind) {
    case 0: k_lens_column<<<blocks, 256, 0, s>>>(X, n, d, column, f); break;
    case 4: k_lens_values<<<blocks, 256, 0, s>>>(values, n, f); break;
    case 1: case 2: case 3:
        k_lens_rows<<<dim3((unsigned)((n + LB - 1) / LB)), dim3(LB), 0, s>>>(X, n, d, kind, dir, f);
        break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_range(const double *f, int64_t n, unsigned long long *keys2, hipStream_t s) {
    int64_t blocks = (n + 255) / 256;
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    k_range<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(f, n, keys2);
    return hipGetLastError();
}

}  // namespace mgpu
