// recheck.hip -- FP64 work on original coordinates: the re-decision of band pairs and the
// helpers of the precision autotuner.
#include "internal.h"

namespace mgpu {

namespace {

// FP64 re-decision of band pairs.  A wave takes its segment's pairs 64 at a
// time: lane l loads pair l's record and the cloud rows of its two slots (so
// these dependent loads cost one round trip per 64 pairs); then the wave
// re-decides them eight at a time (two rounds of four, their row loads
// issued together), sixteen lanes on each pair: lane g of a group sums
// (x_j - y_j)^2 over the 16-byte chunks g, g + 16, ... of the two rows with
// an FMA chain, and the group adds its partials as a tree (four steps, the
// four groups together).  Any summation order is within
// gamma_{d+4} D of the exact value, as is the canonical chain (x_j - y_j in
// FP64, fma in index order), so the two are within 2 gamma_{d+4} D of each
// other and only pairs that close to eps^2 (ties, in practice) need the
// canonical chain itself, which the group's first lane then evaluates.
// Workgroups are dealt to the 8 XCDs in turn; those of one XCD serve
// segments XCD, XCD + 8, ..., RECHECK_WG_PER_SEG of them per segment.
constexpr int RECHECK_WG_PER_SEG = 16;
constexpr int GL = 16;                 // lanes per pair
constexpr int GP = WAVE / GL;          // pairs of one round (a group each)
constexpr int RR = 2;                  // rounds whose row loads are in flight together

__global__ void __launch_bounds__(256) k_recheck(const BandPair *band, const unsigned long long *band_n,
                                                 int64_t band_cap, const float *X,
                                                 int32_t d, const uint32_t *slot_point, Levels lv,
                                                 uint32_t *bitmask, int32_t *count) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int xcd = blockIdx.x & 7, idx = blockIdx.x >> 3;
    const int seg = (idx / RECHECK_WG_PER_SEG) * 8 + xcd;
    const int64_t nw = RECHECK_WG_PER_SEG * (blockDim.x / WAVE);
    const int64_t wid = (int64_t)(idx % RECHECK_WG_PER_SEG) * (blockDim.x / WAVE) + threadIdx.x / WAVE;
    const int64_t n = (int64_t)band_n[seg] < band_cap ? (int64_t)band_n[seg] : band_cap;
    const BandPair *sb = band + (int64_t)seg * band_cap;
    const double u = 0x1.0p-53;
    const double gd = (d + 4) * u / (1.0 - (d + 4) * u);
    const double cf = 4.0 * gd / (1.0 - gd);              // twice the certified gap, for margin
    const int gq = lane / GL, gl = lane % GL;
    const bool vec4 = (d & 3) == 0;                        // rows start on 16-byte boundaries
    for (int64_t c0 = wid * WAVE; c0 < n; c0 += nw * WAVE) {
        const int m = (int)(n - c0 < WAVE ? n - c0 : WAVE);  // pairs of this chunk
        BandPair bp{};
        int px = 0, py = 0;
        if (lane < m) {
            bp = sb[c0 + lane];
            px = (int)slot_point[bp.si];
            py = (int)slot_point[bp.sj];
        }
        const int blo = (int)(uint32_t)bp.bit, bhi = (int)(uint32_t)(bp.bit >> 32);
        for (int g = 0; g < m; g += GP * RR) {
            int kk[RR];
            bool live[RR];
            const float *x[RR], *y[RR];
            double s[RR];
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                const int k = g + r * GP + gq;               // this group's pair in round r
                live[r] = k < m;
                kk[r] = live[r] ? k : g;                     // idle groups repeat the first pair
                x[r] = X + (int64_t)__shfl(px, kk[r], WAVE) * d;
                y[r] = X + (int64_t)__shfl(py, kk[r], WAVE) * d;
                s[r] = 0.0;
            }
            if (vec4) {
#pragma unroll 2
                for (int j = 4 * gl; j < d; j += 4 * GL) {
                    float4 xv[RR], yv[RR];
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        xv[r] = *(const float4 *)(x[r] + j);
                        yv[r] = *(const float4 *)(y[r] + j);
                    }
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        double t = (double)xv[r].x - (double)yv[r].x;
                        s[r] = __builtin_fma(t, t, s[r]);
                        t = (double)xv[r].y - (double)yv[r].y;
                        s[r] = __builtin_fma(t, t, s[r]);
                        t = (double)xv[r].z - (double)yv[r].z;
                        s[r] = __builtin_fma(t, t, s[r]);
                        t = (double)xv[r].w - (double)yv[r].w;
                        s[r] = __builtin_fma(t, t, s[r]);
                    }
                }
            } else {
#pragma unroll 2
                for (int j = gl; j < d; j += GL) {
#pragma unroll
                    for (int r = 0; r < RR; ++r) {
                        const double t = (double)x[r][j] - (double)y[r][j];
                        s[r] = __builtin_fma(t, t, s[r]);
                    }
                }
            }
#pragma unroll
            for (int o = GL / 2; o > 0; o >>= 1)
#pragma unroll
                for (int r = 0; r < RR; ++r) s[r] += __shfl_xor(s[r], o, WAVE);
#pragma unroll
            for (int r = 0; r < RR; ++r) {
                const uint64_t bit =
                    ((uint64_t)(uint32_t)__shfl(bhi, kk[r], WAVE) << 32) | (uint32_t)__shfl(blo, kk[r], WAVE);
                const int level = (int)(bit >> BAND_LEVEL_SHIFT);
                const double E = lv.E[level];
                bool in = s[r] <= E;
                if (fabs(s[r] - E) <= cf * s[r]) {           // a near-tie: the canonical chain decides
                    double D = 0.0;
                    if (gl == 0)
                        for (int32_t j = 0; j < d; ++j) {
                            const double t = (double)x[r][j] - (double)y[r][j];
                            D = __builtin_fma(t, t, D);
                        }
                    in = __shfl(D, lane & ~(GL - 1), WAVE) <= E;
                }
                const int si = __shfl(bp.si, kk[r], WAVE), sj = __shfl(bp.sj, kk[r], WAVE);
                if (live[r] && in && gl == 0) {
                    const uint64_t b = bit & ((1ull << BAND_LEVEL_SHIFT) - 1);
                    uint32_t *bm = bitmask + (uint64_t)level * lv.level_words;
                    int32_t *cn = count + (int64_t)level * lv.level_slots;
                    atomicOr(&bm[b >> 5], 1u << (b & 31u));
                    atomicAdd(&cn[si], 1);
                    atomicAdd(&cn[sj], 1);
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
    if (nseg % 8 != 0) return hipErrorInvalidValue;        // segments are dealt to the 8 XCDs
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
