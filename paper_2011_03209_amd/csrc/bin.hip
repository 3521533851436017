// bin.hip -- pullback sets of the cover and packed distance panels.
//
// Membership (Background section): point i lies in interval k of an axis iff
// lo_k <= f_i <= hi_k.  The endpoint sequences are non-decreasing (lo_k by
// construction, hi_k after clamping to the lens maximum, which no point
// exceeds), so the intervals holding a point form one contiguous index range
// per axis, found by two binary searches.  Each point emits its (element,
// point) pairs in ascending element order; a stable radix sort by element then
// lists every element's members in ascending point order.
//
// Packing copies each member row into a per-slot panel in the matrix-core
// input format (FP32, or BF16/FP16 with an optional low part), scaled by a
// power of two so that every FP32 intermediate stays far from overflow and
// underflow, and computes the per-slot thresholds that let the tile epilogue
// decide "certainly a neighbour" / "certainly not" with two adds and two
// compares per pair.
#include "internal.h"

namespace mgpu {

namespace {

__device__ __forceinline__ int first_ge(const double *a, int n, double f) {
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] >= f) hi = mid; else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ int last_le(const double *a, int n, double f) {
    int lo = 0, hi = n;           // count of entries <= f
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= f) lo = mid + 1; else hi = mid;
    }
    return lo - 1;
}

// *out += the workgroup's sum of v (one atomic per 256-thread workgroup;
// every thread of the workgroup calls it).
__device__ __forceinline__ void block_pair_sum(unsigned long long v, unsigned long long *out) {
    __shared__ unsigned long long part[4];
    for (int o = WAVE / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) part[threadIdx.x / WAVE] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long t = part[0] + part[1] + part[2] + part[3];
        if (t) atomicAdd(out, t);
    }
}

// Per point: its range of intervals on each axis, its number of elements,
// and (pair_sum, optional) the sum over points of C(count, 2), which bounds
// the node pairs that share a point and so the edge builder's work.
__global__ void k_member_count(const double *f0, const double *f1, int64_t n,
                               const double *lo0, const double *hc0, int32_t n0,
                               const double *lo1, const double *hc1, int32_t n1,
                               int32_t *range4, int32_t *count, unsigned long long *pair_sum) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int c = 0;
    if (i < n) {
        const double a = f0[i];
        const int kl0 = first_ge(hc0, n0, a), kh0 = last_le(lo0, n0, a);
        c = kh0 >= kl0 ? kh0 - kl0 + 1 : 0;
        int kl1 = 0, kh1 = 0;
        if (f1) {
            const double b = f1[i];
            kl1 = first_ge(hc1, n1, b);
            kh1 = last_le(lo1, n1, b);
            c *= kh1 >= kl1 ? kh1 - kl1 + 1 : 0;
        }
        range4[4 * i + 0] = kl0;
        range4[4 * i + 1] = kh0;
        range4[4 * i + 2] = kl1;
        range4[4 * i + 3] = kh1;
        count[i] = c;
    }
    // every thread of the workgroup reaches this point (no early return)
    if (pair_sum) block_pair_sum((unsigned long long)c * (unsigned long long)(c > 0 ? c - 1 : 0) / 2, pair_sum);
}

__global__ void k_member_emit(const int32_t *range4, const int64_t *pos, int64_t n, int32_t n1,
                              int two_d, const uint16_t *okey, int key_bits, uint64_t *keys, uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int64_t p = pos[i];
    const int kl0 = range4[4 * i], kh0 = range4[4 * i + 1];
    const int kl1 = two_d ? range4[4 * i + 2] : 0, kh1 = two_d ? range4[4 * i + 3] : 0;
    const uint64_t c = okey ? (uint64_t)okey[i] : 0;
    for (int k0 = kl0; k0 <= kh0; ++k0)
        for (int k1 = kl1; k1 <= kh1; ++k1) {
            keys[p] = ((uint64_t)((int64_t)k0 * (two_d ? n1 : 1) + k1) << key_bits) | c;
            vals[p] = (uint32_t)i;
            ++p;
        }
}

// ------------------------------------------------------------------ packing

// Round to nearest even BF16; results below the smallest normal are flushed
// to zero so the matrix cores never see denormals.
__device__ __forceinline__ float bf16_round(float x, uint16_t *bits) {
    uint32_t u = __float_as_uint(x);
    uint32_t r = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    if ((r & 0x7f800000u) == 0) r = 0;          // zero or denormal
    *bits = (uint16_t)(r >> 16);
    return __uint_as_float(r);
}

__device__ __forceinline__ float fp16_round(float x, uint16_t *bits) {
    _Float16 h = (_Float16)x;                    // round to nearest even
    float hv = (float)h;
    if (fabsf(hv) < 6.103515625e-05f) { h = (_Float16)0.0f; hv = 0.0f; }
    uint16_t b;
    __builtin_memcpy(&b, &h, 2);
    *bits = b;
    return hv;
}

__device__ __forceinline__ double gam(double k) {
    const double u = 0x1.0p-23;                 // covers RNE and truncating accumulators
    return k * u / (1.0 - k * u);
}

// Next float towards +inf / -inf (finite inputs).
__device__ __forceinline__ float next_up(float f) {
    if (f == 0.0f) return __uint_as_float(1u);
    const uint32_t b = __float_as_uint(f);
    return __uint_as_float(f > 0.0f ? b + 1u : b - 1u);
}

__device__ __forceinline__ float next_down(float f) { return -next_up(-f); }

__device__ __forceinline__ float round_up_f(double v) {
    float f = (float)v;
    if ((double)f < v) f = next_up(f);
    return f;
}

__device__ __forceinline__ float round_dn_f(double v) {
    float f = (float)v;
    if ((double)f > v) f = next_down(f);
    return f;
}

// Sixteen lanes per slot (four slots per wave): lane `sub` of a slot handles
// coordinates 4 sub .. 4 sub + 3, then 64 further on, and so on, so a slot's
// loads and its panel stores are contiguous 256-byte runs (one 16-byte load
// and one 8- or 16-byte store per lane), and each cross-lane step of the
// FP64 sums serves four slots at once.
constexpr int PK_LANES = 16;

__global__ void __launch_bounds__(256) k_pack(PackArgs a) {
    const int sub = threadIdx.x & (PK_LANES - 1);
    const int64_t s0 = block_linear() * (blockDim.x / PK_LANES);
    if (s0 >= a.n_slots) return;                           // a padding block of the 2-D grid
    const int64_t s = s0 + threadIdx.x / PK_LANES;
    const bool live = s < a.n_slots;                       // lanes of absent slots still join the shuffles
    const int64_t sl = live ? s : a.n_slots - 1;
    const float *x = a.X + (int64_t)a.slot_point[sl] * a.d;
    const bool split = a.prec == P_BF16X3 || a.prec == P_FP16X3;
    const bool bf = a.prec == P_BF16 || a.prec == P_BF16X3;
    const bool vec = (a.d & 3) == 0;                       // rows start 16-byte aligned
    char *row = (char *)a.panel + s * panel_row_stride(a.prec, a.dp);
    double nx = 0, hh = 0, ll = 0, xt = 0, rr = 0;
    // the power-of-two scale in FP32 when it is a normal float: the product
    // is then the same correctly rounded value as through FP64
    const bool fsc = a.scale >= 0x1.0p-126 && a.scale <= 0x1.0p127;
    const float scf = (float)a.scale;
    for (int j0 = 4 * sub; j0 < a.dp; j0 += 4 * PK_LANES) {   // dp is a multiple of 32
        float v[4];
        if (vec && j0 + 4 <= a.d) {
            const float4 q = *(const float4 *)(x + j0);
            v[0] = q.x; v[1] = q.y; v[2] = q.z; v[3] = q.w;
        } else {
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = j0 + q < a.d ? x[j0 + q] : 0.0f;
        }
        float xs[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xs[q] = fsc ? v[q] * scf : (float)((double)v[q] * a.scale);   // power-of-two scaling
            nx = __builtin_fma((double)xs[q], (double)xs[q], nx);        // the square is exact
        }
        if (a.prec == P_FP32) {
            if (live) *(float4 *)(row + (int64_t)j0 * 4) = make_float4(xs[0], xs[1], xs[2], xs[3]);
            continue;
        }
        uint16_t hb[4], lb[4] = {0, 0, 0, 0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const float h = bf ? bf16_round(xs[q], &hb[q]) : fp16_round(xs[q], &hb[q]);
            double lo = 0.0;
            if (split) {
                const float rem = xs[q] - h;                 // exact in FP32
                lo = (double)(bf ? bf16_round(rem, &lb[q]) : fp16_round(rem, &lb[q]));
            }
            const double hd = (double)h, r = (double)xs[q] - hd - lo;   // exact in FP64
            const double hl = hd + lo;                       // exact; every square below is too
            hh = __builtin_fma(hd, hd, hh);
            ll = __builtin_fma(lo, lo, ll);
            xt = __builtin_fma(hl, hl, xt);
            rr = __builtin_fma(r, r, rr);
        }
        // split rows interleave 16 hi and 16 lo values per group of 16 coordinates
        const int64_t at = split ? (int64_t)(j0 >> 4) * 32 + (j0 & 15) : j0;
        if (live) {
            uint16_t *row16 = (uint16_t *)row;
            *(uint2 *)(row16 + at) = make_uint2(hb[0] | ((uint32_t)hb[1] << 16), hb[2] | ((uint32_t)hb[3] << 16));
            if (split)
                *(uint2 *)(row16 + at + 16) =
                    make_uint2(lb[0] | ((uint32_t)lb[1] << 16), lb[2] | ((uint32_t)lb[3] << 16));
        }
    }
#pragma unroll
    for (int o = PK_LANES / 2; o > 0; o >>= 1) {            // within each slot's 16 lanes
        nx += __shfl_xor(nx, o, WAVE);
        hh += __shfl_xor(hh, o, WAVE);
        ll += __shfl_xor(ll, o, WAVE);
        xt += __shfl_xor(xt, o, WAVE);
        rr += __shfl_xor(rr, o, WAVE);
    }
    if (sub != 0 || !live) return;
    // Per-slot share e_s of the bound |g_ij - x_i.x_j| <= e_i + e_j on the tile's
    // Gram value (every product bound made separable with a*b <= (l a^2 + b^2/l)/2).
    const double K = (double)a.dp;
    double e;
    if (a.prec == P_FP32) {
        e = gam(2 * K + 2) * nx * 0.5;                    // rounded products + sums
    } else if (!split) {
        const double rho = bf ? 0x1.0p-9 : 0x1.0p-12;     // nominal relative residual
        e = gam(K + 2) * hh * 0.5                         // exact products, FP32 sums
            + (rho * hh + rr / rho + rr) * 0.5;           // x.r_y + r_x.y + r_x.r_y
    } else {
        const double rho = bf ? 0x1.0p-17 : 0x1.0p-23;    // residual after hi + lo
        const double rl = bf ? 0x1.0p-8 : 0x1.0p-11;      // |lo| / |hi|
        e = gam(K + 2) * hh * 0.5                         // hi.hi accumulator
            + gam(2 * K + 2) * (rl * hh + ll / rl) * 0.5  // cross accumulator
            + 0x1.0p-23 * xt * 0.5                        // adding the two accumulators
            + ll * 0.5                                    // dropped lo.lo
            + (rho * xt + rr / rho + rr) * 0.5;           // residual beyond hi + lo
    }
    e += 0x1.0p-40 * nx + (3 * K + 8) * 0x1.0p-110;       // FP64 norm / distance rounding, underflow
    for (int t = 0; t < a.n_levels; ++t) {                  // one threshold pair per eps value
        const double Eh = a.E_scaled[t] * 0.5;
        const double A = (nx + 2 * e - Eh) * 0.5;           // g >= A_i + A_j  =>  D <= eps^2
        const double B = (nx - 2 * e - Eh) * 0.5;           // g <  B_i + B_j  =>  D >  eps^2
        a.thrA[(int64_t)t * a.n_slots + s] = round_up_f(A + 0x1.0p-22 * fabs(A));
        a.thrB[(int64_t)t * a.n_slots + s] = round_dn_f(B - 0x1.0p-22 * fabs(B));
    }
    if (a.dbg_norm2) a.dbg_norm2[s] = nx;
    if (a.dbg_e) a.dbg_e[s] = e;
}

}  // namespace

hipError_t launch_member_count(const double *f0, const double *f1, int64_t n,
                               const double *lo0, const double *hc0, int32_t n0,
                               const double *lo1, const double *hc1, int32_t n1,
                               int32_t *range4, int32_t *count, unsigned long long *pair_sum, hipStream_t s) {
    k_member_count<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(
        f0, f1, n, lo0, hc0, n0, lo1, hc1, n1, range4, count, pair_sum);
    return hipGetLastError();
}

hipError_t launch_member_emit(const int32_t *range4, const int64_t *pos, int64_t n, int32_t n1,
                              int two_d, const uint16_t *okey, int key_bits, uint64_t *keys, uint32_t *vals,
                              hipStream_t s) {
    k_member_emit<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(range4, pos, n, n1, two_d,
                                                                         okey, key_bits, keys, vals);
    return hipGetLastError();
}

hipError_t launch_pack(const PackArgs &a, hipStream_t s) {
    if (a.n_slots <= 0) return hipSuccess;
    // sixteen lanes per slot: past 268M slots one grid dimension would
    // exceed 2^32 work-items
    const int64_t blocks = (a.n_slots + 256 / PK_LANES - 1) / (256 / PK_LANES);
    k_pack<<<grid_2d(blocks), dim3(256), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace mgpu
