// recheck.hip -- FP64 work on original coordinates: the re-decision of band pairs and the
// helpers of the precision autotuner.
#include "internal.h"

namespace mgpu {

namespace {

// FP64 re-decision of band pairs.  A wave takes its segment's pairs 64 at a
// time: lane l loads pair l's record and the cloud rows of its two slots (so
// these dependent loads cost one round trip per 64 pairs); then the wave
// re-decides them four at a time, all lanes on each pair with the loads of
// the four issued together.  Lane l sums (x_j - y_j)^2 over j = l, l + 64,
// ... with an FMA chain and the wave adds the partials as a tree.  Any
// summation order is within gamma_{d+4} D of the exact value, as is the
// canonical chain (x_j - y_j in FP64, fma in index order), so the two are
// within 2 gamma_{d+4} D of each other and only pairs that close to eps^2
// (ties, in practice) need the canonical chain itself, which lane 0 then
// evaluates.  Workgroups RECHECK_WG_PER_SEG * g .. + RECHECK_WG_PER_SEG - 1
// serve band segment g.
constexpr int RECHECK_WG_PER_SEG = 16;
constexpr int RG = 4;                  // pairs re-decided together (their row loads in flight at once)

__global__ void __launch_bounds__(256) k_recheck(const BandPair *band, const unsigned long long *band_n,
                                                 int64_t band_cap, const float *X,
                                                 int32_t d, const uint32_t *slot_point, Levels lv,
                                                 uint32_t *bitmask, int32_t *count) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int seg = blockIdx.x / RECHECK_WG_PER_SEG;
    const int64_t nw = RECHECK_WG_PER_SEG * (blockDim.x / WAVE);
    const int64_t wid = (int64_t)(blockIdx.x % RECHECK_WG_PER_SEG) * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int64_t n = (int64_t)band_n[seg] < band_cap ? (int64_t)band_n[seg] : band_cap;
    const BandPair *sb = band + (int64_t)seg * band_cap;
    const double u = 0x1.0p-53;
    const double gd = (d + 4) * u / (1.0 - (d + 4) * u);
    const double cf = 4.0 * gd / (1.0 - gd);              // twice the certified gap, for margin
    for (int64_t c0 = wid * WAVE; c0 < n; c0 += nw * WAVE) {
        const int m = (int)(n - c0 < WAVE ? n - c0 : WAVE);  // pairs of this chunk
        BandPair bp{};
        int px = 0, py = 0;
        if (lane < m) {
            bp = sb[c0 + lane];
            px = (int)slot_point[bp.si];
            py = (int)slot_point[bp.sj];
        }
        for (int g = 0; g < m; g += RG) {
            const int np = m - g < RG ? m - g : RG;
            const float *x[RG], *y[RG];
#pragma unroll
            for (int i = 0; i < RG; ++i) {
                const int k = g + (i < np ? i : 0);          // slots past np repeat the first pair
                x[i] = X + (int64_t)__builtin_amdgcn_readlane(px, k) * d;
                y[i] = X + (int64_t)__builtin_amdgcn_readlane(py, k) * d;
            }
            double s[RG];
#pragma unroll
            for (int i = 0; i < RG; ++i) s[i] = 0.0;
            for (int j0 = 0; j0 < d; j0 += 4 * WAVE) {
                float xv[RG][4], yv[RG][4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int j = j0 + q * WAVE + lane;
                    const int jj = j < d ? j : d - 1;       // in bounds; the term is dropped below
#pragma unroll
                    for (int i = 0; i < RG; ++i) {
                        xv[i][q] = x[i][jj];
                        yv[i][q] = y[i][jj];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool live = j0 + q * WAVE + lane < d;
#pragma unroll
                    for (int i = 0; i < RG; ++i) {
                        const double t = live ? (double)xv[i][q] - (double)yv[i][q] : 0.0;
                        s[i] = __builtin_fma(t, t, s[i]);
                    }
                }
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
#pragma unroll
                for (int i = 0; i < RG; ++i) s[i] += __shfl_xor(s[i], o, WAVE);
#pragma unroll
            for (int i = 0; i < RG; ++i) {
                if (i < np) {
                    const int level = (int)__builtin_amdgcn_readlane((int)(uint32_t)(bp.bit >> BAND_LEVEL_SHIFT), g + i);
                    const double E = lv.E[level];
                    bool in = s[i] <= E;
                    if (fabs(s[i] - E) <= cf * s[i]) {      // a near-tie: the canonical chain decides
                        double D = 0.0;
                        if (lane == 0)
                            for (int32_t j = 0; j < d; ++j) {
                                const double t = (double)x[i][j] - (double)y[i][j];
                                D = __builtin_fma(t, t, D);
                            }
                        in = __shfl(D, 0, WAVE) <= E;
                    }
                    if (in && lane == g + i) {               // the lane holding the pair's record
                        const uint64_t bit = bp.bit & ((1ull << BAND_LEVEL_SHIFT) - 1);
                        uint32_t *bm = bitmask + (uint64_t)level * lv.level_words;
                        int32_t *cn = count + (int64_t)level * lv.level_slots;
                        atomicOr(&bm[bit >> 5], 1u << (bit & 31u));
                        atomicAdd(&cn[bp.si], 1);
                        atomicAdd(&cn[bp.sj], 1);
                    }
                }
            }
        }
    }
}

__global__ void __launch_bounds__(256) k_pair_d64(const int32_t *pa, const int32_t *pb, int64_t np,
                                                  const float *X, int32_t d, double *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= np) return;
    const float *x = X + (int64_t)pa[t] * d;
    const float *y = X + (int64_t)pb[t] * d;
    double D = 0.0;
    for (int32_t j = 0; j < d; ++j) {
        const double u = (double)x[j] - (double)y[j];
        D = __builtin_fma(u, u, D);
    }
    out[t] = D;
}

__global__ void __launch_bounds__(256) k_row_norm2(const int32_t *rows, int64_t nr, const float *X,
                                                   int32_t d, double *out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nr) return;
    const float *x = X + (int64_t)rows[t] * d;
    double s = 0.0;
    for (int32_t j = 0; j < d; ++j) s += (double)x[j] * (double)x[j];
    out[t] = s;
}

}  // namespace

hipError_t launch_recheck(const BandPair *band, const unsigned long long *band_n, int32_t nseg,
                          int64_t band_cap, int64_t nband, const float *X, int32_t d,
                          const uint32_t *slot_point, const Levels &lv, uint32_t *bitmask, int32_t *count,
                          hipStream_t s) {
    if (nband <= 0) return hipSuccess;
    k_recheck<<<dim3((unsigned)(nseg * RECHECK_WG_PER_SEG)), dim3(256), 0, s>>>(band, band_n, band_cap, X, d,
                                                                              slot_point, lv, bitmask, count);
    return hipGetLastError();
}

hipError_t launch_row_norm2(const int32_t *rows, int64_t nr, const float *X, int32_t d,
                            double *out, hipStream_t s) {
    if (nr <= 0) return hipSuccess;
    k_row_norm2<<<dim3((unsigned)((nr + 255) / 256)), dim3(256), 0, s>>>(rows, nr, X, d, out);
    return hipGetLastError();
}

hipError_t launch_pair_d64(const int32_t *pa, const int32_t *pb, int64_t np, const float *X,
                           int32_t d, double *out, hipStream_t s) {
    if (np <= 0) return hipSuccess;
    k_pair_d64<<<dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s>>>(pa, pb, np, X, d, out);
    return hipGetLastError();
}

}  // namespace mgpu
