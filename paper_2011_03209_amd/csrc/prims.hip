// prims.hip -- device-wide exclusive scan and stable LSD radix sort.
//
// Both are written for wave64: block-level scans combine a 64-lane shuffle
// scan with a tiny cross-wave step in LDS, and the radix sort ranks keys
// stably inside each wave with eight ballots per 8-bit digit (lanes whose
// digits agree are found by intersecting the ballot of every digit bit).
#include "internal.h"

namespace mgpu {

namespace {

constexpr int SB = 256;           // threads per block
constexpr int SI = 8;             // items per thread
constexpr int ST = SB * SI;       // items per block

template <typename T>
__device__ __forceinline__ int64_t ld_item(const T *p, int64_t i, int64_t n) {
    return i < n ? (int64_t)p[i] : 0;
}

// Exclusive scan of one value per thread across a 256-thread block.
__device__ int64_t block_exclusive(int64_t v, int64_t *total) {
    __shared__ int64_t wsum[SB / WAVE];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    int64_t inc = v;
#pragma unroll
    for (int o = 1; o < WAVE; o <<= 1) {
        int64_t t = __shfl_up(inc, o, WAVE);
        if (lane >= o) inc += t;
    }
    if (lane == WAVE - 1) wsum[w] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < SB / WAVE; ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    __syncthreads();
    if (total) *total = all;
    return before + inc - v;
}

template <typename T>
__global__ void __launch_bounds__(SB) k_scan_reduce(const T *in, int64_t n, int64_t *part) {
    const int64_t base = (int64_t)blockIdx.x * ST + (int64_t)threadIdx.x * SI;
    int64_t s = 0;
#pragma unroll
    for (int k = 0; k < SI; ++k) s += ld_item(in, base + k, n);
    int64_t tot;
    block_exclusive(s, &tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

// Single block: exclusive scan of the per-block sums, in place.
__global__ void __launch_bounds__(SB) k_scan_parts(int64_t *part, int64_t nb, int64_t *out_total) {
    int64_t carry = 0;
    for (int64_t c0 = 0; c0 < nb; c0 += ST) {
        const int64_t base = c0 + (int64_t)threadIdx.x * SI;
        int64_t v[SI], s = 0;
#pragma unroll
        for (int k = 0; k < SI; ++k) { v[k] = ld_item(part, base + k, nb); s += v[k]; }
        int64_t tot;
        int64_t ex = block_exclusive(s, &tot) + carry;
#pragma unroll
        for (int k = 0; k < SI; ++k) {
            if (base + k < nb) part[base + k] = ex;
            ex += v[k];
        }
        carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) *out_total = carry;
}

template <typename T>
__global__ void __launch_bounds__(SB) k_scan_down(const T *in, int64_t n, const int64_t *part,
                                                  int64_t *out) {
    const int64_t base = (int64_t)blockIdx.x * ST + (int64_t)threadIdx.x * SI;
    int64_t v[SI], s = 0;
#pragma unroll
    for (int k = 0; k < SI; ++k) { v[k] = ld_item(in, base + k, n); s += v[k]; }
    int64_t ex = block_exclusive(s, nullptr) + part[blockIdx.x];
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
}

// The whole scan in one block (n <= ST): one launch instead of three.
template <typename T>
__global__ void __launch_bounds__(SB) k_scan_small(const T *in, int64_t n, int64_t *out) {
    const int64_t base = (int64_t)threadIdx.x * SI;
    int64_t v[SI], s = 0;
#pragma unroll
    for (int k = 0; k < SI; ++k) { v[k] = ld_item(in, base + k, n); s += v[k]; }
    int64_t tot;
    int64_t ex = block_exclusive(s, &tot);
#pragma unroll
    for (int k = 0; k < SI; ++k) {
        if (base + k < n) out[base + k] = ex;
        ex += v[k];
    }
    if (threadIdx.x == 0) out[n] = tot;
}

template <typename T>
hipError_t scan_impl(const T *in, int64_t *out, int64_t n, void *temp, hipStream_t s) {
    int64_t *part = (int64_t *)temp;
    const int64_t nb = (n + ST - 1) / ST;
    if (nb <= 1) {
        k_scan_small<T><<<1, SB, 0, s>>>(in, n, out);
        return hipGetLastError();
    }
    if (nb > 0) {
        k_scan_reduce<T><<<dim3((unsigned)nb), dim3(SB), 0, s>>>(in, n, part);
    }
    k_scan_parts<<<1, SB, 0, s>>>(part, nb, out + n);
    if (nb > 0) {
        k_scan_down<T><<<dim3((unsigned)nb), dim3(SB), 0, s>>>(in, n, part, out);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------ radix sort

__global__ void __launch_bounds__(SB) k_radix_hist(const uint64_t *keys, int64_t n, int shift,
                                                   int32_t *counts, int64_t nb) {
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * ST;
    for (int k = 0; k < SI; ++k) {
        const int64_t i = base + (int64_t)k * SB + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    counts[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// Items of a block are ordered (wave, round, lane): wave w owns the 512 items
// starting at base + 512 w, taken 64 at a time.
__global__ void __launch_bounds__(SB) k_radix_scatter(const uint64_t *keys, const uint32_t *vals,
                                                      int64_t n, int shift, const int64_t *offs,
                                                      int64_t nb, uint64_t *okeys, uint32_t *ovals) {
    __shared__ int32_t wcount[SB / WAVE][256];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    for (int k = threadIdx.x; k < (SB / WAVE) * 256; k += SB) (&wcount[0][0])[k] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * ST + (int64_t)w * (SI * WAVE);
    const uint64_t lt = (1ull << lane) - 1ull;
    int rank[SI];
    int dig[SI];
    uint64_t key[SI];
    uint32_t val[SI];
#pragma unroll
    for (int r = 0; r < SI; ++r) {
        const int64_t i = base + (int64_t)r * WAVE + lane;
        const bool valid = i < n;
        key[r] = valid ? keys[i] : 0;
        val[r] = valid ? vals[i] : 0;
        const int dg = (int)((key[r] >> shift) & 255u);
        dig[r] = dg;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t bb = __ballot((dg >> b) & 1);
            peers &= ((dg >> b) & 1) ? bb : ~bb;
        }
        int before = 0;
        if (valid) before = wcount[w][dg];
        rank[r] = before + __popcll(peers & lt);
        // the lowest lane of each digit group advances the wave's counter
        if (valid && (peers & lt) == 0) wcount[w][dg] = before + __popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {
        const int dg = threadIdx.x;      // 256 threads, one digit each
        int32_t run = 0;
#pragma unroll
        for (int k = 0; k < SB / WAVE; ++k) {
            const int32_t c = wcount[k][dg];
            wcount[k][dg] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < SI; ++r) {
        const int64_t i = base + (int64_t)r * WAVE + lane;
        if (i < n) {
            const int64_t pos = offs[(int64_t)dig[r] * nb + blockIdx.x] + wcount[w][dig[r]] + rank[r];
            okeys[pos] = key[r];
            ovals[pos] = val[r];
        }
    }
}

// The whole sort in one block (n <= ST): every pass ranks the items as
// k_radix_scatter does, with the digit offsets from the block's own counts,
// and scatters them into LDS; the sorted pairs are written back in place.
// One launch instead of five per pass.
__global__ void __launch_bounds__(SB) k_radix_small(uint64_t *keys, uint32_t *vals, int64_t n, int key_bits) {
    __shared__ int32_t wcount[SB / WAVE][256];
    __shared__ int32_t doff[256];
    __shared__ uint64_t sk[ST];
    __shared__ uint32_t sv[ST];
    const int lane = threadIdx.x & (WAVE - 1), w = threadIdx.x / WAVE;
    const int64_t base = (int64_t)w * (SI * WAVE);
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int64_t i = threadIdx.x; i < n; i += SB) {
        sk[i] = keys[i];
        sv[i] = vals[i];
    }
    for (int shift = 0; shift < key_bits; shift += 8) {
        for (int k = threadIdx.x; k < (SB / WAVE) * 256; k += SB) (&wcount[0][0])[k] = 0;
        __syncthreads();                                     // the items (loaded or scattered) are in LDS
        int rank[SI], dig[SI];
        uint64_t key[SI];
        uint32_t val[SI];
#pragma unroll
        for (int r = 0; r < SI; ++r) {
            const int64_t i = base + (int64_t)r * WAVE + lane;
            const bool valid = i < n;
            key[r] = valid ? sk[i] : 0;
            val[r] = valid ? sv[i] : 0;
            const int dg = (int)((key[r] >> shift) & 255u);
            dig[r] = dg;
            uint64_t peers = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const uint64_t bb = __ballot((dg >> b) & 1);
                peers &= ((dg >> b) & 1) ? bb : ~bb;
            }
            int before = 0;
            if (valid) before = wcount[w][dg];
            rank[r] = before + __popcll(peers & lt);
            if (valid && (peers & lt) == 0) wcount[w][dg] = before + __popcll(peers);
            __builtin_amdgcn_wave_barrier();
        }
        __syncthreads();
        int32_t tot = 0;
        {
            const int dg = threadIdx.x;                      // 256 threads, one digit each
#pragma unroll
            for (int k = 0; k < SB / WAVE; ++k) {
                const int32_t c = wcount[k][dg];
                wcount[k][dg] = tot;
                tot += c;
            }
        }
        const int64_t ex = block_exclusive(tot, nullptr);    // (synchronizes the block)
        doff[threadIdx.x] = (int32_t)ex;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < SI; ++r) {
            const int64_t i = base + (int64_t)r * WAVE + lane;
            if (i < n) {
                const int pos = doff[dig[r]] + wcount[w][dig[r]] + rank[r];
                sk[pos] = key[r];
                sv[pos] = val[r];
            }
        }
        __syncthreads();                                     // every scatter done before wcount is cleared
    }
    for (int64_t i = threadIdx.x; i < n; i += SB) {
        keys[i] = sk[i];
        vals[i] = sv[i];
    }
}

__global__ void k_lower_bounds(const uint64_t *keys, int64_t n, int64_t nv, int64_t *out) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > nv) return;
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (keys[mid] < (uint64_t)v) lo = mid + 1; else hi = mid;
    }
    out[v] = lo;
}

}  // namespace

size_t scan_temp_bytes(int64_t n) {
    const int64_t nb = (n + ST - 1) / ST;
    return (size_t)(nb + 8) * sizeof(int64_t);
}

hipError_t launch_scan_i32(const int32_t *in, int64_t *out, int64_t n, void *temp, hipStream_t s) {
    return scan_impl(in, out, n, temp, s);
}
hipError_t launch_scan_i64(const int64_t *in, int64_t *out, int64_t n, void *temp, hipStream_t s) {
    return scan_impl(in, out, n, temp, s);
}
hipError_t launch_scan_u8(const uint8_t *in, int64_t *out, int64_t n, void *temp, hipStream_t s) {
    return scan_impl(in, out, n, temp, s);
}

size_t sort_temp_bytes(int64_t n) {
    const int64_t nb = (n + ST - 1) / ST;
    const int64_t nc = 256 * (nb > 0 ? nb : 1);
    // counts (int32) + offsets (int64, nc + 1) + scan temp
    size_t b = (size_t)nc * sizeof(int32_t);
    b = (b + 255) & ~(size_t)255;
    b += (size_t)(nc + 1) * sizeof(int64_t);
    b = (b + 255) & ~(size_t)255;
    b += scan_temp_bytes(nc);
    return b;
}

hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt,
                            uint32_t *vals_alt, int64_t n, int key_bits, void *temp,
                            bool *result_in_alt, hipStream_t s) {
    *result_in_alt = false;
    if (n <= 1 || key_bits <= 0) return hipSuccess;
    const int64_t nb = (n + ST - 1) / ST;
    if (nb == 1) {                                           // in place, one launch
        k_radix_small<<<1, SB, 0, s>>>(keys, vals, n, key_bits);
        return hipGetLastError();
    }
    const int64_t nc = 256 * nb;
    char *t = (char *)temp;
    int32_t *counts = (int32_t *)t;
    size_t o = ((size_t)nc * sizeof(int32_t) + 255) & ~(size_t)255;
    int64_t *offs = (int64_t *)(t + o);
    o += (size_t)(nc + 1) * sizeof(int64_t);
    o = (o + 255) & ~(size_t)255;
    void *stemp = t + o;
    uint64_t *ki = keys, *ko = keys_alt;
    uint32_t *vi = vals, *vo = vals_alt;
    bool alt = false;
    for (int shift = 0; shift < key_bits; shift += 8) {
        k_radix_hist<<<dim3((unsigned)nb), dim3(SB), 0, s>>>(ki, n, shift, counts, nb);
        hipError_t e = launch_scan_i32(counts, offs, nc, stemp, s);
        if (e != hipSuccess) return e;
        k_radix_scatter<<<dim3((unsigned)nb), dim3(SB), 0, s>>>(ki, vi, n, shift, offs, nb, ko, vo);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t *tk = ki; ki = ko; ko = tk;
        uint32_t *tv = vi; vi = vo; vo = tv;
        alt = !alt;
    }
    *result_in_alt = alt;
    return hipSuccess;
}

namespace {

__global__ void k_iota_u32(uint32_t *out, int64_t n) {
    const int64_t i = block_linear() * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint32_t)i;
}

// *out = max(*out, max_i in[i]) (in[i] >= 0): a wave maximum, then one
// atomic per wave.
__global__ void k_max_i32(const int32_t *in, int64_t n, int32_t *out) {
    const int64_t i = block_linear() * blockDim.x + threadIdx.x;
    int v = i < n ? in[i] : 0;
    for (int o = WAVE / 2; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, WAVE));
    if ((threadIdx.x & (WAVE - 1)) == 0 && v > 0) atomicMax(out, v);
}

}  // namespace

hipError_t launch_iota_u32(uint32_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_iota_u32<<<grid_2d((n + 255) / 256), dim3(256), 0, s>>>(out, n);
    return hipGetLastError();
}

hipError_t launch_max_i32(const int32_t *in, int64_t n, int32_t *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_max_i32<<<grid_2d((n + 255) / 256), dim3(256), 0, s>>>(in, n, out);
    return hipGetLastError();
}

hipError_t launch_lower_bounds(const uint64_t *keys, int64_t n, int64_t nv, int64_t *out,
                               hipStream_t s) {
    const int64_t cnt = nv + 1;
    k_lower_bounds<<<dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s>>>(keys, n, nv, out);
    return hipGetLastError();
}

}  // namespace mgpu
