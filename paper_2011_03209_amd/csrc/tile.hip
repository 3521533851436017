// tile.hip -- eps-neighbourhood of every cover element by matrix-core Gram tiles.
//
// DBSCAN (Ester et al.) needs, inside each pullback set, every pair's
// decision D(x, y) <= eps^2; the paper names this all-pairs query as the cost
// centre of DBSCAN-based mapper (Scalability section) and precomputes
// distance matrices per interval.  Here the per-interval matrix is never
// stored: with D = |x|^2 + |y|^2 - 2 x.y the only dense contraction is the
// Gram block X_I X_J^T, computed on the matrix cores one 128 x 128 tile pair
// (I <= J) at a time, and each pair leaves one bit.
//
// Decisions are certified: the per-slot thresholds A_s, B_s (packing stage)
// bound every rounding and representation error of the tile's Gram value g,
// so g >= A_i + A_j proves D <= eps^2 and g < B_i + B_j proves D > eps^2.
// Pairs in between (the band) are appended to a list and re-decided with the
// canonical FP64 distance by k_recheck, so the bitmask is exact whatever the
// tile precision.
//
// Layout: a workgroup of 4 waves owns one tile pair; wave (wm, wn) owns the
// 64 x 64 quadrant as 2 x 2 blocks of 32 x 32 accumulators.  K runs over
// double-buffered LDS slabs of 128 bytes (64 bytes per panel for hi/lo
// splits) per row, rows padded by 16 bytes so 16-byte fragment reads from 8
// consecutive rows hit distinct banks.  In a 32x32 accumulator lane l holds
// column l%32 of rows 8(v/4) + 4(l/32) + v%4 (v = 0..15), so a ballot of
// register v yields two 32-bit row words of the bitmask directly.
//
// Bitmask: one 128 x 128-bit block (128 rows x 4 words) per tile pair, in the
// element's pair order p = J(J+1)/2 + I; bit (r, c) means pair
// (I*128 + r, J*128 + c) are neighbours.  Diagonal blocks keep only r <= c,
// so every unordered pair is stored once.
#include "internal.h"

// v_writelane_b32: set lane `lane` of `old` to the wave-uniform `val`.
extern "C" __device__ int lane_write(int val, int lane, int old) __asm("llvm.amdgcn.writelane.i32");

namespace mgpu {

namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

constexpr int NT = 256;              // threads per workgroup

template <int PREC> struct Cfg;
template <> struct Cfg<P_FP32>   { static constexpr int ESZ = 4, KC = 32, PANELS = 1; };
template <> struct Cfg<P_BF16>   { static constexpr int ESZ = 2, KC = 64, PANELS = 1; };
template <> struct Cfg<P_FP16>   { static constexpr int ESZ = 2, KC = 64, PANELS = 1; };
template <> struct Cfg<P_BF16X3> { static constexpr int ESZ = 2, KC = 32, PANELS = 2; };
template <> struct Cfg<P_FP16X3> { static constexpr int ESZ = 2, KC = 32, PANELS = 2; };

template <int PREC> struct Lay {
    static constexpr int RB = Cfg<PREC>::KC * Cfg<PREC>::ESZ;   // bytes of a row per slab
    static constexpr int CPR = RB / 16;                         // 16-byte chunks per row
    static constexpr int PANEL_BYTES = TILE * RB;                // one operand panel
    static constexpr int STAGE_BYTES = 2 * Cfg<PREC>::PANELS * PANEL_BYTES;   // A and B
    static constexpr int CPT = TILE * CPR / NT;                  // chunks per thread per panel
    static constexpr int NREG = 2 * Cfg<PREC>::PANELS * CPT;
};

// LDS rows are unpadded; the 16-byte chunks of row r are permuted by an XOR
// with swz(r).  16-byte reads of one chunk column by 8 (32-bank) or 16
// (64-bank) consecutive rows, and writes of consecutive chunks of consecutive
// rows, then all fall in distinct banks.
template <int CPR> __device__ __forceinline__ int swz(int r) {
    if constexpr (CPR == 8) return (r + (r >> 3)) & 7;
    else return ((r >> 1) ^ (r >> 3)) & 3;
}

template <int CPR> __device__ __forceinline__ int loff(int r, int c) {
    return (r * CPR + (c ^ swz<CPR>(r))) * 16;
}

// Per-thread copy plan of one tile.  The row panels of the two sides (and of
// the hi/lo halves of a split) start at wave-uniform addresses; a thread
// moves chunk c of rows r_q (q < CPT) of each, found at a 32-bit offset from
// that start.  Rows past the element are clamped to its last row (masked in
// the epilogue).
template <int PREC> struct Feed {
    const char *base[2 * Cfg<PREC>::PANELS];
    uint32_t voff[2][Lay<PREC>::CPT];
    int dst[Lay<PREC>::CPT];
};

template <int PREC>
__device__ __forceinline__ void feed_setup(const TileArgs &a, const TilePos &tl, Feed<PREC> &f) {
    using L = Lay<PREC>;
    const uint32_t rowb = (uint32_t)a.dp * Cfg<PREC>::ESZ;
#pragma unroll
    for (int side = 0; side < 2; ++side) {
        const int64_t r0 = (int64_t)(side == 0 ? tl.I : tl.J) * TILE;
        const int64_t nrow = tl.ne - r0;
#pragma unroll
        for (int pnl = 0; pnl < Cfg<PREC>::PANELS; ++pnl)
            f.base[side * Cfg<PREC>::PANELS + pnl] =
                (const char *)(pnl == 0 ? a.panel_hi : a.panel_lo) + (tl.slot0 + r0) * (int64_t)rowb;
#pragma unroll
        for (int q = 0; q < L::CPT; ++q) {
            const int idx = q * NT + threadIdx.x;
            const int r = idx / L::CPR, c = idx % L::CPR;
            const int rr = r < nrow ? r : (int)(nrow - 1);
            f.voff[side][q] = (uint32_t)rr * rowb + (uint32_t)(c * 16);
        }
    }
#pragma unroll
    for (int q = 0; q < L::CPT; ++q) {
        const int idx = q * NT + threadIdx.x;
        f.dst[q] = loff<L::CPR>(idx / L::CPR, idx % L::CPR);
    }
}

template <int PREC>
__device__ __forceinline__ void gload(const Feed<PREC> &f, uint32_t koff, u32x4 *reg) {
    using L = Lay<PREC>;
#pragma unroll
    for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int pnl = 0; pnl < Cfg<PREC>::PANELS; ++pnl) {
            const char *bk = f.base[side * Cfg<PREC>::PANELS + pnl] + koff;
#pragma unroll
            for (int q = 0; q < L::CPT; ++q)
                reg[(side * Cfg<PREC>::PANELS + pnl) * L::CPT + q] = *(const u32x4 *)(bk + f.voff[side][q]);
        }
}

template <int PREC>
__device__ __forceinline__ void lstore(char *stage, const Feed<PREC> &f, const u32x4 *reg) {
    using L = Lay<PREC>;
#pragma unroll
    for (int sp = 0; sp < 2 * Cfg<PREC>::PANELS; ++sp)
#pragma unroll
        for (int q = 0; q < L::CPT; ++q)
            *(u32x4 *)(stage + sp * L::PANEL_BYTES + f.dst[q]) = reg[sp * L::CPT + q];
}

template <int PREC> struct Acc {
    f32x16 c[2][2];
    f32x16 x[2][2];   // cross-term accumulator of hi/lo splits
};

// FIRST: the first slab, whose products start the accumulators (MFMA with a
// zero addend, so the accumulators need no clearing).
template <int PREC, bool FIRST>
__device__ __forceinline__ void compute_stage(const char *stage, Acc<PREC> &acc, int wm, int wn) {
    using L = Lay<PREC>;
    const f32x16 zero = {};
    constexpr int CPR = L::CPR;
    const int lane = threadIdx.x & (WAVE - 1);
    const int li = lane & 31, lg = lane >> 5;
    const char *Ah = stage;
    const char *Bh = stage + Cfg<PREC>::PANELS * L::PANEL_BYTES;
    if constexpr (PREC == P_FP32) {
        // 16 bytes = 4 k values per lane; MFMA t of a step takes element t, so
        // lane group g supplies k = 8 ss + 4 g + t for both operands
#pragma unroll
        for (int ss = 0; ss < Cfg<PREC>::KC / 8; ++ss) {
            f32x4 av[2], bv[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                av[b] = *(const f32x4 *)(Ah + loff<CPR>(wm * 64 + b * 32 + li, 2 * ss + lg));
                bv[b] = *(const f32x4 *)(Bh + loff<CPR>(wn * 64 + b * 32 + li, 2 * ss + lg));
            }
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                    for (int bn = 0; bn < 2; ++bn)
                        acc.c[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                            av[bm][t], bv[bn][t], FIRST && ss == 0 && t == 0 ? zero : acc.c[bm][bn], 0, 0, 0);
        }
    } else {
        constexpr bool SPLIT = Cfg<PREC>::PANELS == 2;
        const char *Al = Ah + L::PANEL_BYTES;
        const char *Bl = Bh + L::PANEL_BYTES;
#pragma unroll
        for (int ks = 0; ks < Cfg<PREC>::KC / 16; ++ks) {
            u32x4 ah[2], bh[2], al[2], bl[2];
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                const int oa = loff<CPR>(wm * 64 + b * 32 + li, 2 * ks + lg);
                const int ob = loff<CPR>(wn * 64 + b * 32 + li, 2 * ks + lg);
                ah[b] = *(const u32x4 *)(Ah + oa);
                bh[b] = *(const u32x4 *)(Bh + ob);
                if constexpr (SPLIT) {
                    al[b] = *(const u32x4 *)(Al + oa);
                    bl[b] = *(const u32x4 *)(Bl + ob);
                }
            }
            const bool z0 = FIRST && ks == 0;
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int bn = 0; bn < 2; ++bn) {
                    if constexpr (PREC == P_BF16 || PREC == P_BF16X3) {
                        acc.c[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, ah[bm]), __builtin_bit_cast(bf16x8, bh[bn]),
                            z0 ? zero : acc.c[bm][bn], 0, 0, 0);
                        if constexpr (SPLIT) {
                            acc.x[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, ah[bm]), __builtin_bit_cast(bf16x8, bl[bn]),
                                z0 ? zero : acc.x[bm][bn], 0, 0, 0);
                            acc.x[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                                __builtin_bit_cast(bf16x8, al[bm]), __builtin_bit_cast(bf16x8, bh[bn]),
                                acc.x[bm][bn], 0, 0, 0);
                        }
                    } else {
                        acc.c[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                            __builtin_bit_cast(f16x8, ah[bm]), __builtin_bit_cast(f16x8, bh[bn]),
                            z0 ? zero : acc.c[bm][bn], 0, 0, 0);
                        if constexpr (SPLIT) {
                            acc.x[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                __builtin_bit_cast(f16x8, ah[bm]), __builtin_bit_cast(f16x8, bl[bn]),
                                z0 ? zero : acc.x[bm][bn], 0, 0, 0);
                            acc.x[bm][bn] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                                __builtin_bit_cast(f16x8, al[bm]), __builtin_bit_cast(f16x8, bh[bn]),
                                acc.x[bm][bn], 0, 0, 0);
                        }
                    }
                }
        }
    }
}

struct EpiShared {
    __attribute__((aligned(16))) float thrA[2 * TILE];
    __attribute__((aligned(16))) float thrB[2 * TILE];
    __attribute__((aligned(16))) uint32_t words[TILE * 4];
    int32_t colcnt[4][TILE];   // column counts, one partial per 32-row band of lanes
};

// Decisions of one 32 x 32 accumulator block: the row words of its bitmask
// go to LDS, the lane's column count is added to colc, and the result says
// whether the block has band pairs.  FULL: the block lies inside the element
// and off the diagonal, so no bounds or triangle masks are needed.
template <int PREC, bool FULL, bool DEBUG>
__device__ __forceinline__ bool epi_block(const TileArgs &a, const TilePos &tl, EpiShared &es,
                                          const Acc<PREC> &acc, int bm, int bn, int wm, int wn, int &colc) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int li = lane & 31, lg = lane >> 5;
    const bool diag = tl.I == tl.J;
    const int cl = wn * 64 + bn * 32 + li;                  // column within the tile
    const int64_t gc = (int64_t)tl.J * TILE + cl;          // element-local column
    const float Aj = es.thrA[TILE + cl], Bj = es.thrB[TILE + cl];
    const int r0 = wm * 64 + bm * 32 + 4 * lg;             // register v holds row r0 + 8(v/4) + v%4
    f32x4 TA[4], TB[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        TA[q] = *(const f32x4 *)&es.thrA[r0 + 8 * q];
        TB[q] = *(const f32x4 *)&es.thrB[r0 + 8 * q];
    }
    int word = 0;                                          // lane li (< 32): row li of the block
    uint64_t anyband = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        float g = acc.c[bm][bn][v];
        if constexpr (Cfg<PREC>::PANELS == 2) g = g + acc.x[bm][bn][v];
        bool in, band;
        if constexpr (FULL) {
            in = g >= TA[v >> 2][v & 3] + Aj;
            band = !(g < TB[v >> 2][v & 3] + Bj);           // band once the "in" pairs are removed
            colc += in ? 1 : 0;
        } else {
            const int rl = r0 + 8 * (v >> 2) + (v & 3);
            const int64_t gr = (int64_t)tl.I * TILE + rl;
            const bool valid = gr < tl.ne && gc < tl.ne && (!diag || rl <= cl);
            const bool self = diag && rl == cl;
            in = valid && (self || g >= TA[v >> 2][v & 3] + Aj);
            band = valid && !in && !(g < TB[v >> 2][v & 3] + Bj);
            colc += (in && !self) ? 1 : 0;
            if constexpr (DEBUG) {
                if (gr < tl.ne && gc < tl.ne) {
                    a.debug_g[gr * a.debug_ld + gc] = g;
                    a.debug_g[gc * a.debug_ld + gr] = g;
                }
            }
        }
        const uint64_t ib = __ballot(in);
        // the low half of the ballot is row 8(v/4) + v%4, the high half the row 4 below
        word = lane_write((int)(uint32_t)ib, 8 * (v >> 2) + (v & 3), word);
        word = lane_write((int)(uint32_t)(ib >> 32), 8 * (v >> 2) + 4 + (v & 3), word);
        anyband |= __ballot(band) & ~ib;
        asm volatile("" : "+s"(anyband));                 // fold now: keeps no masks live
    }
    if (lane < 32) es.words[(wm * 64 + bm * 32 + li) * 4 + wn * 2 + bn] = (uint32_t)word;
    return anyband != 0;
}

// Band pairs of one block -> FP64 recheck list (rare; wave-aggregated append).
template <int PREC>
__device__ __forceinline__ void epi_band(const TileArgs &a, const TilePos &tl, const EpiShared &es,
                                      const Acc<PREC> &acc, int bm, int bn, int wm, int wn) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int li = lane & 31, lg = lane >> 5;
    const bool diag = tl.I == tl.J;
    const int cl = wn * 64 + bn * 32 + li;
    const int64_t gc = (int64_t)tl.J * TILE + cl;
    const float Aj = es.thrA[TILE + cl], Bj = es.thrB[TILE + cl];
    const int r0 = wm * 64 + bm * 32 + 4 * lg;
    // the decisions are recomputed in each pass rather than kept (keeps the
    // common path free of their registers)
    auto band_at = [&](int v) -> bool {
        const int rl = r0 + 8 * (v >> 2) + (v & 3);
        const int64_t gr = (int64_t)tl.I * TILE + rl;
        float g = acc.c[bm][bn][v];
        if constexpr (Cfg<PREC>::PANELS == 2) g = g + acc.x[bm][bn][v];
        asm volatile("" : "+v"(g));
        const bool valid = gr < tl.ne && gc < tl.ne && (!diag || rl <= cl);
        const bool self = diag && rl == cl;
        const bool in = valid && (self || g >= es.thrA[rl] + Aj);
        return valid && !in && !(g < es.thrB[rl] + Bj);
    };
    int nb = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) nb += __popcll(__ballot(band_at(v)));
    unsigned long long base = 0;
    if (lane == 0) base = atomicAdd(a.band_n, (unsigned long long)nb);
    base = __shfl(base, 0, WAVE);
    const uint64_t lt = (1ull << lane) - 1ull;
    int before = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int rl = r0 + 8 * (v >> 2) + (v & 3);
        const int64_t gr = (int64_t)tl.I * TILE + rl;
        const bool band = band_at(v);
        const uint64_t bb = __ballot(band);
        if (band) {
            const int64_t idx = (int64_t)base + before + __popcll(bb & lt);
            if (idx < a.band_cap) {
                BandPair bp;
                bp.si = (int32_t)(tl.slot0 + gr);
                bp.sj = (int32_t)(tl.slot0 + gc);
                bp.bit = ((uint64_t)tl.blk * TILE_WORDS + (uint64_t)(rl * 4 + (cl >> 5))) * 32u
                         + (uint64_t)(cl & 31);
                a.band[idx] = bp;
            }
        }
        before += __popcll(bb);
    }
}

template <int PREC, bool DEBUG>
__device__ void process_tile(const TileArgs &a, const TilePos &tl, char *stages, EpiShared &es) {
    using L = Lay<PREC>;
    const int w = threadIdx.x / WAVE;
    const int wm = w >> 1, wn = w & 1;
    const bool diag = tl.I == tl.J;

    // K loop: double-buffered LDS slabs, the next slab's global loads in
    // flight while the current one feeds the matrix cores
    const int nst = a.dp / Cfg<PREC>::KC;
    Feed<PREC> feed;
    feed_setup<PREC>(a, tl, feed);
    u32x4 reg[L::NREG];
    gload<PREC>(feed, 0, reg);
    // thresholds of the tile's rows and columns (read in the epilogue)
    {
        const int t = threadIdx.x;
        const int64_t rb = (t < TILE ? (int64_t)tl.I : (int64_t)tl.J) * TILE + (t & (TILE - 1));
        const int64_t slot = tl.slot0 + (rb < tl.ne ? rb : tl.ne - 1);
        const float ta = a.thrA[slot], tb = a.thrB[slot];
        es.thrA[t] = ta;
        es.thrB[t] = tb;
    }
    lstore<PREC>(stages, feed, reg);
    __syncthreads();
    Acc<PREC> acc;
    if (nst > 1) gload<PREC>(feed, L::RB, reg);
    compute_stage<PREC, true>(stages, acc, wm, wn);
    if (nst > 1) lstore<PREC>(stages + L::STAGE_BYTES, feed, reg);
    __syncthreads();
    for (int st = 1; st < nst; ++st) {
        char *cur = stages + (st & 1) * L::STAGE_BYTES;
        if (st + 1 < nst) gload<PREC>(feed, (uint32_t)(st + 1) * L::RB, reg);
        compute_stage<PREC, false>(cur, acc, wm, wn);
        if (st + 1 < nst) lstore<PREC>(stages + ((st + 1) & 1) * L::STAGE_BYTES, feed, reg);
        __syncthreads();
    }

    // ---------------------------------------------------------------- epilogue
    const bool full = !diag && (int64_t)(tl.I + 1) * TILE <= tl.ne && (int64_t)(tl.J + 1) * TILE <= tl.ne;
    bool hb[2][2];
    int colc[2] = {0, 0};
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn) {
            if (!DEBUG && full) hb[bm][bn] = epi_block<PREC, true, false>(a, tl, es, acc, bm, bn, wm, wn, colc[bn]);
            else hb[bm][bn] = epi_block<PREC, false, DEBUG>(a, tl, es, acc, bm, bn, wm, wn, colc[bn]);
        }
    {
        const int lane = threadIdx.x & (WAVE - 1);
        es.colcnt[wm * 2 + (lane >> 5)][wn * 64 + (lane & 31)] = colc[0];
        es.colcnt[wm * 2 + (lane >> 5)][wn * 64 + 32 + (lane & 31)] = colc[1];
    }
#pragma unroll
    for (int bm = 0; bm < 2; ++bm)
#pragma unroll
        for (int bn = 0; bn < 2; ++bn)
            if (hb[bm][bn]) epi_band<PREC>(a, tl, es, acc, bm, bn, wm, wn);
    __syncthreads();
    // bitmask block (2 KB, coalesced) and neighbour counts: a row's count is
    // the popcount of its four words, a column's the sum of its partials
    {
        uint32_t *dst = a.bitmask + (uint64_t)tl.blk * TILE_WORDS;
        const int t = threadIdx.x;
        *(uint2 *)(dst + 2 * t) = *(const uint2 *)(es.words + 2 * t);
        if (t < TILE) {
            const int64_t r = (int64_t)tl.I * TILE + t;
            const u32x4 wv = *(const u32x4 *)(es.words + 4 * t);
            const int c = __popc(wv.x) + __popc(wv.y) + __popc(wv.z) + __popc(wv.w);
            if (r < tl.ne && c) atomicAdd(&a.count[tl.slot0 + r], c);
        } else {
            const int cc = t - TILE;
            const int64_t gc = (int64_t)tl.J * TILE + cc;
            const int c = es.colcnt[0][cc] + es.colcnt[1][cc] + es.colcnt[2][cc] + es.colcnt[3][cc];
            if (gc < tl.ne && c) atomicAdd(&a.count[tl.slot0 + gc], c);
        }
    }
    __syncthreads();
}

template <int PREC, bool DEBUG>
__global__ void __launch_bounds__(NT, 2) k_tiles(TileArgs a) {
    __shared__ __attribute__((aligned(16))) char stages[2 * Lay<PREC>::STAGE_BYTES];
    __shared__ EpiShared es;
    // XCD-aware order: the hardware deals workgroups round-robin to the 8
    // XCDs, so consecutive tile pairs (which share row panels) are mapped to
    // one XCD and its L2.
    const int64_t G = gridDim.x;
    const int64_t per = (G + 7) / 8;
    const int64_t item = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    if (item >= a.tt.n_items) return;
    const TilePos tl = tile_lookup(a.tt, item);
    process_tile<PREC, DEBUG>(a, tl, stages, es);
}

// FP64 re-decision of band pairs, one pair per wave at a time.  The lanes
// read the two rows with coalesced loads and sum (x_j - y_j)^2 in FP64 as a
// tree; that value is within 2 gamma_{d+4} D of the canonical sequential
// chain, so only pairs closer than that to eps^2 (ties, in practice) need
// the canonical chain itself, which lane 0 then evaluates in order.
// Persistent form: a fixed grid (a few workgroups per CU) drains the tile
// pairs through eight atomic counters, one per XCD slice of the item order
// (largest elements first).  A workgroup starts on the slice of the XCD it
// was dealt to and then helps the others; it leaves when every slice is
// exhausted, so the grid always drains.
template <int PREC>
__global__ void __launch_bounds__(NT, 2) k_tiles_persistent(TileArgs a) {
    __shared__ __attribute__((aligned(16))) char stages[2 * Lay<PREC>::STAGE_BYTES];
    __shared__ EpiShared es;
    __shared__ int64_t next;
    const int64_t n = a.tt.n_items;
    const int64_t per = (n + 7) / 8;
    const int x0 = blockIdx.x % 8;
    for (int k = 0; k < 8; ++k) {
        const int x = (x0 + k) % 8;
        const int64_t lo = (int64_t)x * per;
        const int64_t hi = lo + per < n ? lo + per : n;
        while (true) {
            if (threadIdx.x == 0) next = lo + (int64_t)atomicAdd(&a.queue[x], 1u);
            __syncthreads();
            const int64_t item = next;
            __syncthreads();
            if (item >= hi) break;
            const TilePos tl = tile_lookup(a.tt, item);
            process_tile<PREC, false>(a, tl, stages, es);
        }
    }
}

__global__ void __launch_bounds__(256) k_recheck(const BandPair *band, int64_t nband, const float *X,
                                                 int32_t d, const uint32_t *slot_point, double E,
                                                 uint32_t *bitmask, int32_t *count) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
    const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / WAVE;
    const double u = 0x1.0p-53;
    const double gd = (d + 4) * u / (1.0 - (d + 4) * u);
    const double cf = 4.0 * gd / (1.0 - gd);              // twice the certified gap, for margin
    for (int64_t b = wid; b < nband; b += nw) {
        const BandPair bp = band[b];
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

__global__ void k_build_items(TileTable tt, TileItem *items) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= tt.n_items) return;
    const TilePos p = tile_decode(tt, i);
    TileItem q;
    q.e = p.e;
    q.I = p.I;
    q.J = p.J;
    q.ne = (int32_t)p.ne;
    q.slot0 = p.slot0;
    q.blk = p.blk;
    items[i] = q;
}

template <int PREC>
hipError_t launch_t(const TileArgs &a, hipStream_t s) {
    if (a.tt.n_items <= 0) return hipSuccess;
    if (a.grid > 0 && !a.debug_g) {
        k_tiles_persistent<PREC><<<dim3((unsigned)a.grid), dim3(NT), 0, s>>>(a);
        return hipGetLastError();
    }
    const int64_t G = 8 * ((a.tt.n_items + 7) / 8);
    if (a.debug_g) k_tiles<PREC, true><<<dim3((unsigned)G), dim3(NT), 0, s>>>(a);
    else k_tiles<PREC, false><<<dim3((unsigned)G), dim3(NT), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

int tile_grid_size(int prec, int64_t n_items) {
    (void)prec;
    return (int)(8 * ((n_items + 7) / 8));
}

hipError_t launch_tiles(int prec, const TileArgs &a, hipStream_t s) {
    switch (prec) {
    case P_FP32: return launch_t<P_FP32>(a, s);
    case P_BF16: return launch_t<P_BF16>(a, s);
    case P_BF16X3: return launch_t<P_BF16X3>(a, s);
    case P_FP16: return launch_t<P_FP16>(a, s);
    case P_FP16X3: return launch_t<P_FP16X3>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_build_items(const TileTable &tt, TileItem *items, hipStream_t s) {
    if (tt.n_items <= 0) return hipSuccess;
    k_build_items<<<dim3((unsigned)((tt.n_items + 255) / 256)), dim3(256), 0, s>>>(tt, items);
    return hipGetLastError();
}

hipError_t launch_recheck(const BandPair *band, int64_t nband, const float *X, int32_t d,
                          const uint32_t *slot_point, double E, uint32_t *bitmask,
                          int32_t *count, hipStream_t s) {
    if (nband <= 0) return hipSuccess;
    int64_t blocks = (nband + 3) / 4;
    if (blocks > 32768) blocks = 32768;
    k_recheck<<<dim3((unsigned)blocks), dim3(256), 0, s>>>(band, nband, X, d, slot_point, E, bitmask, count);
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
