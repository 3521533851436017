// recheck.hip -- FP64 work on original coordinates: the re-decision of band pairs and the
// helpers of the precision autotuner.
#include "internal.h"

namespace mgpu {

namespace {

// FP64 re-decision of band pairs, one pair per wave at a time.  The lanes
// read the two rows with coalesced loads and sum (x_j - y_j)^2 in FP64 as a
// tree; that value is within 2 gamma_{d+4} D of the canonical sequential
// chain, so only pairs closer than that to eps^2 (ties, in practice) need
// the canonical chain itself, which lane 0 then evaluates in order.
// Workgroups RECHECK_WG_PER_SEG * g .. + RECHECK_WG_PER_SEG - 1 serve band
// segment g; their waves take the segment's pairs in turn.
constexpr int RECHECK_WG_PER_SEG = 8;

__global__ void __launch_bounds__(256) k_recheck(const BandPair *band, const unsigned long long *band_n,
                                                 int64_t band_cap, const float *X,
                                                 int32_t d, const uint32_t *slot_point, double E,
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
    for (int64_t b = wid; b < n; b += nw) {
        const BandPair bp = sb[b];
        const float *x = X + (int64_t)slot_point[bp.si] * d;
        const float *y = X + (int64_t)slot_point[bp.sj] * d;
        double part = 0.0;
        for (int32_t j = lane; j < d; j += WAVE) {
            const double t = (double)x[j] - (double)y[j];
            part = __builtin_fma(t, t, part);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) part += __shfl_xor(part, o, WAVE);
        bool in;
        if (fabs(part - E) > cf * part) {
            in = part <= E;
        } else {
            double D = 0.0;                                 // canonical chain, in order
            if (lane == 0)
                for (int32_t j = 0; j < d; ++j) {
                    const double t = (double)x[j] - (double)y[j];
                    D = __builtin_fma(t, t, D);
                }
            D = __shfl(D, 0, WAVE);
            in = D <= E;
        }
        if (in && lane == 0) {
            atomicOr(&bitmask[bp.bit >> 5], 1u << (bp.bit & 31u));
            atomicAdd(&count[bp.si], 1);
            atomicAdd(&count[bp.sj], 1);
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
                          const uint32_t *slot_point, double E, uint32_t *bitmask, int32_t *count,
                          hipStream_t s) {
    if (nband <= 0) return hipSuccess;
    k_recheck<<<dim3((unsigned)(nseg * RECHECK_WG_PER_SEG)), dim3(256), 0, s>>>(band, band_n, band_cap, X, d,
                                                                              slot_point, E, bitmask, count);
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
