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
// Layout: a workgroup of 8 waves owns one tile pair; wave (wm, wn) owns rows
// 64 wm .. + 63 and columns 32 wn .. + 31 as 2 x 1 blocks of 32 x 32
// accumulators.  K runs over double-buffered LDS stages filled by LDS-direct
// loads.  In a 32x32 accumulator lane l holds column l%32 of rows
// 8(v/4) + 4(l/32) + v%4 (v = 0..15), so a ballot of register v yields two
// 32-bit row words of the bitmask directly.
//
// Bitmask: one 128 x 128-bit block (128 rows x 4 words) per tile pair, in the
// element's supertile order; bit (r, c) means pair (I*128 + r, J*128 + c) are
// neighbours.  Diagonal blocks keep only r <= c,
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

constexpr int NTG = 512;             // threads per workgroup (8 waves)

// Per precision: 16-bit or FP32 panel values, one or two (hi/lo) terms.
template <int PREC> struct Cfg;
template <> struct Cfg<P_FP32>   { static constexpr int PANELS = 1; };
template <> struct Cfg<P_BF16>   { static constexpr int PANELS = 1; };
template <> struct Cfg<P_FP16>   { static constexpr int PANELS = 1; };
template <> struct Cfg<P_BF16X3> { static constexpr int PANELS = 2; };
template <> struct Cfg<P_FP16X3> { static constexpr int PANELS = 2; };

__device__ __forceinline__ uint32_t lds_addr(const void *p) {
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) char *)p;
}

// LDS-direct loads: M0 holds the wave's LDS destination (set in the same
// statement; nothing else in these kernels uses M0).  Completion is tracked
// by hand with vmcnt: the compiler does not see these loads.
__device__ __forceinline__ void lds_load16(uint32_t lds, const char *sbase, uint32_t voff) {
    asm volatile("s_mov_b32 m0, %0\n\tglobal_load_lds_dwordx4 %1, %2"
                 :: "s"(__builtin_amdgcn_readfirstlane(lds)), "v"(voff), "s"(sbase) : "memory");
}
// Wait until at most N vector memory operations of this wave are in flight.
template <int N> __device__ __forceinline__ void vm_wait() { asm volatile("s_waitcnt vmcnt(%0)" :: "n"(N) : "memory"); }

// Workgroup barrier over LDS traffic only: the wave's own LDS accesses are
// complete, global memory operations may still be in flight.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// The lane index through an empty asm: values derived from it inside a loop
// body are recomputed there instead of being hoisted into registers that
// would stay live across the whole loop.
__device__ __forceinline__ int lane_id_here() {
    int l = (int)(threadIdx.x & (WAVE - 1));
    asm volatile("" : "+v"(l));
    return l;
}

// A wave's accumulators: two blocks of 32 x 32 (64 x 32 pairs).
template <int PREC> struct Acc {
    f32x16 c[2];
    f32x16 x[2];       // cross-term accumulator of hi/lo splits
};

// ------------------------------------------------ one tile pair per workgroup
// A stage is 128 bytes of every row of both sides (A rows 0..127, then B
// rows): FP32 values 32 s .. + 31, BF16/FP16 values 64 s .. + 63, or for the
// splits two groups of 16 hi then 16 lo values, exactly as in the panel row.
// Chunk c (16 bytes) of stage row r sits at LDS offset r 128 + 16 (c ^ swz(r))
// with swz(r) = (r >> 1) & 7, chosen by measurement on gfx950 (bank-conflict
// counter of a probe kernel): the operand reads, one chunk column of 32
// consecutive rows per half-wave, are then free of bank conflicts.
constexpr int GROW = 128;                     // bytes of a row per stage
constexpr int GSTAGE = 2 * TILE * GROW;       // 32 KB

__device__ __forceinline__ int goff(int r, int c) { return r * GROW + ((c ^ ((r >> 1) & 7)) << 4); }

// LDS-direct plan of one wave for one tile: wave w fills stage rows
// 32 w .. + 31 (side w / 4) with four 1 KB loads of 8 rows; lane l of load i
// writes chunk position l % 8 of stage row 32 w + 8 i + l / 8, so it reads the
// global chunk that belongs there.  Rows past the element are clamped to its
// last row (masked in the epilogue).
struct GridFeed {
    const char *sbase;                        // the side's first row, stage 0
    uint32_t vo[4];
};

__device__ __forceinline__ void grid_setup(const TileArgs &a, const TilePos &tl, int w, int lane,
                                           uint32_t stride, GridFeed &f) {
    const int side = w >> 2;
    const int64_t r0 = (int64_t)(side ? tl.J : tl.I) * TILE;
    const int64_t nrow = tl.ne - r0;                        // rows of this side in the element (>= 1)
    f.sbase = (const char *)a.panel + (tl.slot0 + r0) * (int64_t)stride;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int sr = (w & 3) * 32 + i * 8 + (lane >> 3);  // side row
        const int lr = w * 32 + i * 8 + (lane >> 3);        // stage row
        const int c = (lane & 7) ^ ((lr >> 1) & 7);
        f.vo[i] = (uint32_t)(sr < nrow ? sr : (int)(nrow - 1)) * stride + (uint32_t)(c << 4);
    }
}

__device__ __forceinline__ void grid_issue(const GridFeed &f, uint32_t stage_lds, int w, uint32_t koff) {
#pragma unroll
    for (int i = 0; i < 4; ++i) lds_load16(stage_lds + (uint32_t)((w * 4 + i) * 1024), f.sbase + koff, f.vo[i]);
}

// A stage's operands of one wave (rows 64 wm .. + 63 of A, 32 wn .. + 31 of B):
//   FP32, BF16, FP16: v[3 h + b] = A block b, v[3 h + 2] = B, chunk 2 h + lane / 32;
//   splits: v[6 ks + 2 b + l] = A block b, v[6 ks + 4 + l] = B, chunk 4 ks + 2 l + lane / 32
//           (l = 0 hi, 1 lo).
struct GridOps {
    u32x4 v[12];
};

template <int PREC>
__device__ __forceinline__ void grid_read(const char *stage, GridOps &o, int wm, int wn) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int li = lane & 31, lg = lane >> 5;
    const int ra0 = wm * 64 + li, ra1 = ra0 + 32, rb = TILE + wn * 32 + li;
    if constexpr (Cfg<PREC>::PANELS == 1) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
            o.v[3 * h + 0] = *(const u32x4 *)(stage + goff(ra0, 2 * h + lg));
            o.v[3 * h + 1] = *(const u32x4 *)(stage + goff(ra1, 2 * h + lg));
            o.v[3 * h + 2] = *(const u32x4 *)(stage + goff(rb, 2 * h + lg));
        }
    } else {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const int c = 4 * ks + 2 * l + lg;
                o.v[6 * ks + l] = *(const u32x4 *)(stage + goff(ra0, c));
                o.v[6 * ks + 2 + l] = *(const u32x4 *)(stage + goff(ra1, c));
                o.v[6 * ks + 4 + l] = *(const u32x4 *)(stage + goff(rb, c));
            }
    }
}

// The stage's products into the accumulators (FIRST: the tile's first stage,
// whose products start them: a zero addend, so they need no clearing).
template <int PREC, bool FIRST>
__device__ __forceinline__ void grid_mfma(const GridOps &o, Acc<PREC> &acc) {
    const f32x16 zero = {};
    if constexpr (PREC == P_FP32) {
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int t = 0; t < 4; ++t)
#pragma unroll
                for (int bm = 0; bm < 2; ++bm)
                    acc.c[bm] = __builtin_amdgcn_mfma_f32_32x32x2f32(
                        __builtin_bit_cast(f32x4, o.v[3 * h + bm])[t], __builtin_bit_cast(f32x4, o.v[3 * h + 2])[t],
                        FIRST && h == 0 && t == 0 ? zero : acc.c[bm], 0, 0, 0);
    } else if constexpr (Cfg<PREC>::PANELS == 1) {
#pragma unroll
        for (int h = 0; h < 4; ++h)
#pragma unroll
            for (int bm = 0; bm < 2; ++bm) {
                const f32x16 c = FIRST && h == 0 ? zero : acc.c[bm];
                if constexpr (PREC == P_BF16)
                    acc.c[bm] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, o.v[3 * h + bm]), __builtin_bit_cast(bf16x8, o.v[3 * h + 2]), c,
                        0, 0, 0);
                else
                    acc.c[bm] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                        __builtin_bit_cast(f16x8, o.v[3 * h + bm]), __builtin_bit_cast(f16x8, o.v[3 * h + 2]), c,
                        0, 0, 0);
            }
    } else {
#pragma unroll
        for (int ks = 0; ks < 2; ++ks)
#pragma unroll
            for (int bm = 0; bm < 2; ++bm) {
                const u32x4 ah = o.v[6 * ks + 2 * bm], al = o.v[6 * ks + 2 * bm + 1];
                const u32x4 bh = o.v[6 * ks + 4], bl = o.v[6 * ks + 5];
                const bool z = FIRST && ks == 0;
                if constexpr (PREC == P_BF16X3) {
                    acc.c[bm] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, ah), __builtin_bit_cast(bf16x8, bh), z ? zero : acc.c[bm], 0, 0, 0);
                    acc.x[bm] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, ah), __builtin_bit_cast(bf16x8, bl), z ? zero : acc.x[bm], 0, 0, 0);
                    acc.x[bm] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, al), __builtin_bit_cast(bf16x8, bh), acc.x[bm], 0, 0, 0);
                } else {
                    acc.c[bm] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                        __builtin_bit_cast(f16x8, ah), __builtin_bit_cast(f16x8, bh), z ? zero : acc.c[bm], 0, 0, 0);
                    acc.x[bm] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                        __builtin_bit_cast(f16x8, ah), __builtin_bit_cast(f16x8, bl), z ? zero : acc.x[bm], 0, 0, 0);
                    acc.x[bm] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                        __builtin_bit_cast(f16x8, al), __builtin_bit_cast(f16x8, bh), acc.x[bm], 0, 0, 0);
                }
            }
    }
}

// acc + this lane's bit of a wave mask (the mask as the carry-in of an add):
// one instruction, and the mask is consumed at once instead of being kept
// until the block's end.
__device__ __forceinline__ int add_lane_bit(int acc, uint64_t mask) {
    int r;
    uint64_t carry;
    asm("v_addc_co_u32_e64 %0, %1, 0, %2, %3" : "=v"(r), "=s"(carry) : "v"(acc), "s"(mask));
    return r;
}

// 2 acc + this lane's bit of a wave mask: the bit shifted in at the bottom.
__device__ __forceinline__ uint32_t shift_in_lane_bit(uint32_t acc, uint64_t mask) {
    uint32_t r;
    uint64_t carry;
    asm("v_addc_co_u32_e64 %0, %1, %2, %2, %3" : "=v"(r), "=s"(carry) : "v"(acc), "s"(mask));
    return r;
}

// LV: eps values (levels) the workgroup can serve; the decisions of one
// level at a time go through words and colcnt.
template <int LV> struct EpiShared {
    __attribute__((aligned(16))) float thrA[LV][2 * TILE];
    __attribute__((aligned(16))) float thrB[LV][2 * TILE];
    __attribute__((aligned(16))) uint32_t words[TILE * 4];    // bitmask block: 4 words per row
    uint8_t colcnt[4][TILE];   // column counts, one partial per 32-row band of lanes (<= 32)
};

// Bits j >= k of a 32-bit word, and bit k alone (none when k is outside
// 0 .. 31).
__device__ __forceinline__ uint32_t bits_from(int k) { return k <= 0 ? ~0u : (k >= 32 ? 0u : ~0u << k); }
__device__ __forceinline__ uint32_t bit_at(int k) { return (k >= 0 && k < 32) ? 1u << k : 0u; }

// Decisions of one 32 x 32 accumulator block (its 16 Gram values per lane in
// gv): the row words of its bitmask and of its band pairs go to LDS, and the
// lane's column count is added to colc.  FULL: the block lies inside the
// element and off the diagonal, so no bounds or triangle masks are needed.
// Otherwise (a diagonal or ragged tile pair) the same compares are masked
// with wave-uniform words: the rows and columns inside the element, on the
// diagonal only columns at or past the row, and the pair of a point with
// itself always in.  DEBUG also stores every Gram value.
template <bool FULL, bool DEBUG, int LV>
__device__ __forceinline__ void epi_block(const TileArgs &a, const TilePos &tl, EpiShared<LV> &es, int lv,
                                          const f32x16 &gv, int bm, int wm, int wn, int &colc, uint32_t &bmask) {
    const int lane = lane_id_here();
    const int li = lane & 31, lg = lane >> 5;
    const bool diag = tl.I == tl.J;
    const int cl = wn * 32 + li;                            // column within the tile
    const int64_t gc = (int64_t)tl.J * TILE + cl;          // element-local column
    const float Aj = es.thrA[lv][TILE + cl], Bj = es.thrB[lv][TILE + cl];
    const int r0 = wm * 64 + bm * 32 + 4 * lg;             // register v holds row r0 + 8(v/4) + v%4
    f32x4 TA[4], TB[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        TA[q] = *(const f32x4 *)&es.thrA[lv][r0 + 8 * q];
        TB[q] = *(const f32x4 *)&es.thrB[lv][r0 + 8 * q];
    }
    // masked blocks: rows of tile I inside the element, and the columns
    // wn * 32 .. + 31 of tile J inside it (lane bits)
    const int rbase = wm * 64 + bm * 32, cbase = wn * 32;
    int rows = TILE;
    uint32_t colok = ~0u;
    if constexpr (!FULL && !DEBUG) {
        const int64_t rv = tl.ne - (int64_t)tl.I * TILE, cv = tl.ne - (int64_t)tl.J * TILE - cbase;
        rows = (int)(rv < TILE ? rv : TILE);
        colok = cv >= 32 ? ~0u : (cv <= 0 ? 0u : (1u << cv) - 1u);
    }
    int word = 0;                                          // lane li (< 32): row li of the block
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const float g = gv[v];
        uint64_t ib, bb, cm;                               // in, band, column-count lanes
        if constexpr (FULL) {
            ib = __ballot(g >= TA[v >> 2][v & 3] + Aj);
            bb = __ballot(!(g < TB[v >> 2][v & 3] + Bj)) & ~ib;   // band once the "in" pairs are removed
            cm = ib;
        } else if constexpr (!DEBUG) {
            const int rlo = rbase + 8 * (v >> 2) + (v & 3), rhi = rlo + 4;   // rows of lanes 0-31, 32-63
            const uint32_t vlo = rlo < rows ? colok & (diag ? bits_from(rlo - cbase) : ~0u) : 0u;
            const uint32_t vhi = rhi < rows ? colok & (diag ? bits_from(rhi - cbase) : ~0u) : 0u;
            const uint64_t valid = ((uint64_t)vhi << 32) | vlo;
            const uint64_t self = diag ? (((uint64_t)bit_at(rhi - cbase) << 32) | bit_at(rlo - cbase)) : 0ull;
            ib = (__ballot(g >= TA[v >> 2][v & 3] + Aj) | self) & valid;
            bb = __ballot(!(g < TB[v >> 2][v & 3] + Bj)) & valid & ~ib;
            cm = ib & ~self;
        } else {
            const int rl = r0 + 8 * (v >> 2) + (v & 3);
            const int64_t gr = (int64_t)tl.I * TILE + rl;
            const bool valid = gr < tl.ne && gc < tl.ne && (!diag || rl <= cl);
            const bool self = diag && rl == cl;
            const bool in = valid && (self || g >= TA[v >> 2][v & 3] + Aj);
            const bool band = valid && !in && !(g < TB[v >> 2][v & 3] + Bj);
            if (gr < tl.ne && gc < tl.ne) {
                a.debug_g[gr * a.debug_ld + gc] = g;
                a.debug_g[gc * a.debug_ld + gr] = g;
            }
            ib = __ballot(in);
            bb = __ballot(band);
            cm = __ballot(in && !self);
        }
        colc = add_lane_bit(colc, cm);
        // the low half of a ballot is row 8(v/4) + v%4, the high half the row 4 below
        word = lane_write((int)(uint32_t)ib, 8 * (v >> 2) + (v & 3), word);
        word = lane_write((int)(uint32_t)(ib >> 32), 8 * (v >> 2) + 4 + (v & 3), word);
        // band pairs: the lane's own bit, shifted into its band mask
        bmask = shift_in_lane_bit(bmask, bb);
    }
    if (lane < 32) es.words[(wm * 64 + bm * 32 + li) * 4 + wn] = (uint32_t)word;
    // one block at a time: interleaving the blocks' compares would keep many
    // 64-bit ballot masks live and spill scalar registers
    __builtin_amdgcn_sched_barrier(0);
}

// The band pairs of tile row t (its band words bw) at level lv -> FP64
// recheck list, in segment blockIdx.x % nseg (no single counter is shared by
// the whole launch).  The macro form appends from its workgroups; the tile
// pair form leaves band masks that k_band_collect turns into records.
__device__ __forceinline__ void band_append(const TileArgs &a, const TilePos &tl, int t, u32x4 bw, int lv) {
    const int n = __popc(bw.x) + __popc(bw.y) + __popc(bw.z) + __popc(bw.w);
    const int seg = (int)(blockIdx.x % (unsigned)a.nseg);
    int64_t idx = (int64_t)atomicAdd(&a.band_n[seg], (unsigned long long)n);
    const int64_t gr = (int64_t)tl.I * TILE + t;
    for (int j = 0; j < 4; ++j) {
        uint32_t m = bw[j];
        while (m) {
            const int b = __ffs(m) - 1;
            m &= m - 1;
            if (idx < a.band_cap) {
                const int cl = 32 * j + b;
                BandPair bp;
                bp.si = (int32_t)(tl.slot0 + gr);
                bp.sj = (int32_t)(tl.slot0 + (int64_t)tl.J * TILE + cl);
                bp.bit = (((uint64_t)tl.blk * TILE_WORDS + (uint64_t)(t * 4 + j)) * 32u + (uint64_t)b) |
                         ((uint64_t)lv << BAND_LEVEL_SHIFT);
                a.band[(int64_t)seg * a.band_cap + idx] = bp;
            }
            ++idx;
        }
    }
}

// The Gram values of accumulator block bm (wave-uniform), selected without
// indexing the accumulator array by a run-time value.
template <int PREC>
__device__ __forceinline__ f32x16 acc_block(const Acc<PREC> &acc, int bm) {
    return bm == 1 ? acc.c[1] : acc.c[0];
}


// Per level: decisions of the wave's two accumulator blocks, then (after a
// barrier) the level's 2 KB bitmask block and neighbour counts: a row's count
// is the popcount of its four words, a column's the sum of its partials.
template <int PREC, bool DEBUG, int LV>
__device__ __forceinline__ void tile_epilogue(const TileArgs &a, const TilePos &tl, Acc<PREC> &acc,
                                              EpiShared<LV> &es, int wm, int wn) {
    if constexpr (Cfg<PREC>::PANELS == 2) {                 // Gram value = hi.hi + cross terms
#pragma unroll
        for (int bm = 0; bm < 2; ++bm) acc.c[bm] = acc.c[bm] + acc.x[bm];
    }
    const bool diag = tl.I == tl.J;
    const bool full = !diag && (int64_t)(tl.I + 1) * TILE <= tl.ne && (int64_t)(tl.J + 1) * TILE <= tl.ne;
    const int nlev = LV == 1 ? 1 : a.n_levels;
#pragma unroll 1
    for (int lv = 0; lv < nlev; ++lv) {
        if (lv > 0) lds_barrier();                          // the previous level's words are stored
        int colc = 0;
        uint32_t bmask = 0;                                 // block 0 ends in bits 31 .. 16, block 1 in 15 .. 0
        if constexpr (!DEBUG) {
            if (full) {
#pragma unroll
                for (int bm = 0; bm < 2; ++bm)
                    epi_block<true, false, LV>(a, tl, es, lv, acc.c[bm], bm, wm, wn, colc, bmask);
            } else if constexpr (LV == 1) {                 // diagonal or ragged tiles: masked
#pragma unroll
                for (int bm = 0; bm < 2; ++bm)
                    epi_block<false, false, LV>(a, tl, es, lv, acc.c[bm], bm, wm, wn, colc, bmask);
            } else {                                        // (one copy in the multi-level kernel)
#pragma unroll 1
                for (int bm = 0; bm < 2; ++bm)
                    epi_block<false, false, LV>(a, tl, es, lv, acc_block(acc, bm), bm, wm, wn, colc, bmask);
            }
        } else {
#pragma unroll 1
            for (int bm = 0; bm < 2; ++bm)
                epi_block<false, true, LV>(a, tl, es, lv, acc_block(acc, bm), bm, wm, wn, colc, bmask);
        }
        const int lane = lane_id_here();
        // the band masks of the tile pair: one word per lane of each wave,
        // turned into band records by k_band_collect
        a.bandmask[(uint64_t)lv * a.level_words + (uint64_t)tl.blk * TILE_WORDS + (threadIdx.x & ~(WAVE - 1)) + lane] =
            bmask;
        es.colcnt[wm * 2 + (lane >> 5)][wn * 32 + (lane & 31)] = (uint8_t)colc;
        lds_barrier();
        const int t = (threadIdx.x & ~(WAVE - 1)) + lane;
        if (t < 2 * TILE) {
            uint32_t *dst = a.bitmask + (uint64_t)lv * a.level_words + (uint64_t)tl.blk * TILE_WORDS;
            int32_t *cnt = a.count + (int64_t)lv * a.level_slots + tl.slot0;
            *(uint2 *)(dst + 2 * t) = *(const uint2 *)(es.words + 2 * t);
            if (t < TILE) {
                const int64_t r = (int64_t)tl.I * TILE + t;
                const u32x4 wv = *(const u32x4 *)(es.words + 4 * t);
                const int c = __popc(wv.x) + __popc(wv.y) + __popc(wv.z) + __popc(wv.w);
                if (r < tl.ne && c) atomicAdd(&cnt[r], c);
            } else {
                const int cc = t - TILE;
                const int64_t gc = (int64_t)tl.J * TILE + cc;
                const int c = (int)es.colcnt[0][cc] + es.colcnt[1][cc] + es.colcnt[2][cc] + es.colcnt[3][cc];
                if (gc < tl.ne && c) atomicAdd(&cnt[gc], c);
            }
        }
    }
}

// One tile pair by eight waves: wave (wm, wn) owns rows 64 wm .. + 63 and
// columns 32 wn .. + 31 (two 32 x 32 accumulator blocks).  Double-buffered
// stages filled by LDS-direct loads: the next stage loads while the current
// one feeds the matrix cores.
template <int PREC, bool DEBUG, int LV>
__device__ void process_tile(const TileArgs &a, const TilePos &tl, char *stages, EpiShared<LV> &es) {
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wm = w >> 2, wn = w & 3;
    const uint32_t stride = (uint32_t)panel_row_stride(PREC, a.dp);
    const int nst = (int)(panel_row_bytes(PREC, a.dp) / GROW);   // >= 2
    const uint32_t st_lds = lds_addr(stages);
    GridFeed feed;
    grid_setup(a, tl, w, lane, stride, feed);
    grid_issue(feed, st_lds, w, 0);
    // thresholds of the tile's rows and columns at every level (read in the epilogue)
    if (threadIdx.x < 2 * TILE) {
        const int t = threadIdx.x;
        const int64_t rw = (t < TILE ? (int64_t)tl.I : (int64_t)tl.J) * TILE + (t & (TILE - 1));
        const int64_t slot = tl.slot0 + (rw < tl.ne ? rw : tl.ne - 1);
#pragma unroll
        for (int lv = 0; lv < LV; ++lv) {
            if (lv == 0 || lv < a.n_levels) {
                const float ta = a.thrA[lv * a.level_slots + slot], tb = a.thrB[lv * a.level_slots + slot];
                es.thrA[lv][t] = ta;
                es.thrB[lv][t] = tb;
            }
        }
    }
    Acc<PREC> acc;
    GridOps ops;
#pragma unroll 1
    for (int st = 0; st < nst; ++st) {
        vm_wait<0>();                                       // this wave's part of stage st has landed
        lds_barrier();                                      // ... everyone's; stage st - 1 fully read
        if (st + 1 < nst) grid_issue(feed, st_lds + (uint32_t)(((st + 1) & 1) * GSTAGE), w, (uint32_t)(st + 1) * GROW);
        grid_read<PREC>(stages + (st & 1) * GSTAGE, ops, wm, wn);
        if (st == 0) grid_mfma<PREC, true>(ops, acc);
        else grid_mfma<PREC, false>(ops, acc);
    }
    tile_epilogue<PREC, DEBUG, LV>(a, tl, acc, es, wm, wn);
}

// LV = 1: one eps value; LV = MAX_LEVELS: up to that many (a parameter sweep
// served by one pass over the tiles).
template <int PREC, bool DEBUG, int LV>
__global__ void __launch_bounds__(NTG, 2) k_tiles(TileArgs a) {
    __shared__ __attribute__((aligned(1024))) char stages[2 * GSTAGE];
    __shared__ EpiShared<LV> es;
    // XCD-aware order: the hardware deals workgroups round-robin to the 8
    // XCDs, so consecutive tile pairs (which share row panels) are mapped to
    // one XCD and its L2.  G: the logical workgroups, one per item, rounded
    // up to a multiple of 8 (the 2-D grid may hold a few more).
    const int64_t G = 8 * ((a.tt.n_items + 7) / 8);
    const int64_t bl = block_linear();
    if (bl >= G) return;
    const int64_t per = G / 8;
    const int64_t item = (bl % 8) * per + bl / 8;
    if (item >= a.tt.n_items) return;
    const TilePos tl = tile_lookup(a.tt, item);
    process_tile<PREC, DEBUG, LV>(a, tl, stages, es);
}

// ------------------------------------------------ one macro tile per workgroup
// A macro item pairs 256-row blocks P <= Q of one element: up to four tile
// pairs (2P + a, 2Q + b).  Eight waves; wave (wm, wn) owns rows 128 wm .. +127
// and columns 64 wn .. + 63 of the 256 x 256 product, i.e. half of tile pair
// (a, b) = (wm, wn / 2), as 4 x 2 blocks of 32 x 32 accumulators.  Per 16-wide
// K step a wave reads six operands from LDS for eight products (the tile
// pair form reads three for two), so the LDS traffic per product halves, and
// the per-workgroup work of thresholds, counts and the output pass is spread
// over four tile pairs.  Single 16-bit products only (128 accumulator
// registers); one workgroup per CU (128 KB of stages).
//
// Stage layout as in the tile pair form (128 bytes of each row, the same
// chunk swizzle): stage rows 0 .. 255 are the P side, 256 .. 511 the Q side.
constexpr int MSTAGE = 2 * MTILE * GROW;       // 64 KB

struct MacroShared {
    __attribute__((aligned(16))) float thrA[2 * MTILE];
    __attribute__((aligned(16))) float thrB[2 * MTILE];
    __attribute__((aligned(16))) uint32_t words[4][TILE * 4];    // bitmask block of each tile pair
    __attribute__((aligned(16))) uint32_t bwords[4][TILE * 4];   // its band pairs, same layout
    uint8_t colcnt[4][2][TILE];   // column counts, one partial per half-wave (<= 64 each)
};

// LDS-direct plan of one wave for one stage: wave w fills stage rows
// 64 w .. + 63 (side w / 4) with eight 1 KB loads of 8 rows; rows past the
// element are clamped to its last row (masked in the epilogue).
struct MacroFeed {
    const char *sbase;
    uint32_t vo[8];
};

__device__ __forceinline__ void macro_setup(const TileArgs &a, const MacroItem &mi, int w, int lane,
                                            uint32_t stride, MacroFeed &f) {
    const int side = w >> 2;
    const int64_t r0 = (int64_t)(side ? mi.Q : mi.P) * MTILE;
    const int64_t nrow = (int64_t)mi.ne - r0;                // rows of this side in the element (>= 1)
    f.sbase = (const char *)a.panel + (mi.slot0 + r0) * (int64_t)stride;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int sr = (w & 3) * 64 + i * 8 + (lane >> 3);  // side row
        const int lr = w * 64 + i * 8 + (lane >> 3);        // stage row
        const int c = (lane & 7) ^ ((lr >> 1) & 7);
        f.vo[i] = (uint32_t)(sr < nrow ? sr : (int)(nrow - 1)) * stride + (uint32_t)(c << 4);
    }
}

__device__ __forceinline__ void macro_issue(const MacroFeed &f, uint32_t stage_lds, int w, uint32_t koff) {
#pragma unroll
    for (int i = 0; i < 8; ++i) lds_load16(stage_lds + (uint32_t)((w * 8 + i) * 1024), f.sbase + koff, f.vo[i]);
}

struct MacroAcc {
    f32x16 c[4][2];
};

// One stage (four 16-wide K steps) of a wave's products.
template <int PREC, bool FIRST>
__device__ __forceinline__ void macro_mfma(const char *stage, MacroAcc &acc, int wm, int wn) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int li = lane & 31, lg = lane >> 5;
    const f32x16 zero = {};
#pragma unroll
    for (int h = 0; h < 4; ++h) {
        u32x4 va[4], vb[2];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) va[rb] = *(const u32x4 *)(stage + goff(wm * 128 + rb * 32 + li, 2 * h + lg));
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
            vb[cb] = *(const u32x4 *)(stage + goff(MTILE + wn * 64 + cb * 32 + li, 2 * h + lg));
#pragma unroll
        for (int rb = 0; rb < 4; ++rb)
#pragma unroll
            for (int cb = 0; cb < 2; ++cb) {
                const f32x16 c = FIRST && h == 0 ? zero : acc.c[rb][cb];
                if constexpr (PREC == P_BF16)
                    acc.c[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                        __builtin_bit_cast(bf16x8, va[rb]), __builtin_bit_cast(bf16x8, vb[cb]), c, 0, 0, 0);
                else
                    acc.c[rb][cb] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                        __builtin_bit_cast(f16x8, va[rb]), __builtin_bit_cast(f16x8, vb[cb]), c, 0, 0, 0);
            }
    }
}

// Decisions of accumulator block (rb, cb) of wave (wm, wn) in tile pair
// (I, J): row words of its bitmask and band pairs to LDS, the lane's column
// count returned.  FULL: the tile pair lies inside the element and off the
// diagonal (no masks).
template <bool FULL>
__device__ __forceinline__ int macro_block(MacroShared &ms, int sub, int I, int J, int64_t ne, const f32x16 &gv,
                                           int rb, int cb, int wm, int wn) {
    const int lane = lane_id_here();
    const int li = lane & 31, lg = lane >> 5;
    const bool diag = I == J;
    const int cl = (wn & 1) * 64 + cb * 32 + li;            // column within the tile pair
    const int64_t gc = (int64_t)J * TILE + cl;              // element-local column
    const float Aj = ms.thrA[MTILE + wn * 64 + cb * 32 + li], Bj = ms.thrB[MTILE + wn * 64 + cb * 32 + li];
    const int r0 = rb * 32 + 4 * lg;                        // register v holds row r0 + 8(v/4) + v%4
    f32x4 TA[4], TB[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        TA[q] = *(const f32x4 *)&ms.thrA[wm * TILE + r0 + 8 * q];
        TB[q] = *(const f32x4 *)&ms.thrB[wm * TILE + r0 + 8 * q];
    }
    int word = 0, bword = 0, colc = 0;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const float g = gv[v];
        bool in, band;
        uint64_t cm;                                        // pairs counted for the column
        if constexpr (FULL) {
            in = g >= TA[v >> 2][v & 3] + Aj;
            band = !(g < TB[v >> 2][v & 3] + Bj);
            cm = __ballot(in);
        } else {
            const int rl = r0 + 8 * (v >> 2) + (v & 3);
            const int64_t gr = (int64_t)I * TILE + rl;
            const bool valid = gr < ne && gc < ne && (!diag || rl <= cl);
            const bool self = diag && rl == cl;
            in = valid && (self || g >= TA[v >> 2][v & 3] + Aj);
            band = valid && !in && !(g < TB[v >> 2][v & 3] + Bj);
            cm = __ballot(in && !self);
        }
        colc = add_lane_bit(colc, cm);
        const uint64_t ib = __ballot(in);
        word = lane_write((int)(uint32_t)ib, 8 * (v >> 2) + (v & 3), word);
        word = lane_write((int)(uint32_t)(ib >> 32), 8 * (v >> 2) + 4 + (v & 3), word);
        const uint64_t bb = __ballot(band) & ~ib;           // written without a branch (see epi_block)
        bword = lane_write((int)(uint32_t)bb, 8 * (v >> 2) + (v & 3), bword);
        bword = lane_write((int)(uint32_t)(bb >> 32), 8 * (v >> 2) + 4 + (v & 3), bword);
    }
    if (lane < 32) {
        const int at = (rb * 32 + li) * 4 + (wn & 1) * 2 + cb;
        ms.words[sub][at] = (uint32_t)word;
        ms.bwords[sub][at] = (uint32_t)bword;
    }
    // one block at a time: interleaving the blocks' compares would keep many
    // 64-bit ballot masks live and spill scalar registers
    __builtin_amdgcn_sched_barrier(0);
    return colc;
}

__device__ __forceinline__ int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// The workgroup's item in scalar registers (it is the same for every lane;
// the LDS-direct loads need their base address in scalar registers).
__device__ __forceinline__ MacroItem uniform_item(const MacroItem &m) {
    MacroItem r;
    r.e = __builtin_amdgcn_readfirstlane(m.e);
    r.P = __builtin_amdgcn_readfirstlane(m.P);
    r.Q = __builtin_amdgcn_readfirstlane(m.Q);
    r.ne = __builtin_amdgcn_readfirstlane(m.ne);
    r.slot0 = uniform64(m.slot0);
#pragma unroll
    for (int k = 0; k < 4; ++k) r.blk[k] = uniform64(m.blk[k]);
    r.pad = 0;
    return r;
}

template <int PREC>
__global__ void __launch_bounds__(NTG, 1) k_tiles_macro(TileArgs a) {
    __shared__ __attribute__((aligned(1024))) char stages[2 * MSTAGE];
    __shared__ MacroShared ms;
    // XCD-aware order as in k_tiles: consecutive macro items on one XCD
    const int64_t G = 8 * ((a.n_mitems + 7) / 8);
    const int64_t bl = block_linear();
    if (bl >= G) return;
    const int64_t per = G / 8;
    const int64_t item = (bl % 8) * per + bl / 8;
    if (item >= a.n_mitems) return;
    const MacroItem mi = uniform_item(a.mitems[item]);
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wm = w >> 2, wn = w & 3;
    const uint32_t stride = (uint32_t)panel_row_stride(PREC, a.dp);
    const int nst = (int)(panel_row_bytes(PREC, a.dp) / GROW);   // >= 2
    const uint32_t st_lds = lds_addr(stages);
    MacroFeed feed;
    macro_setup(a, mi, w, lane, stride, feed);
    macro_issue(feed, st_lds, w, 0);
    {   // thresholds of the macro rows (P side) and columns (Q side)
        const int t = threadIdx.x;
        const int64_t rw = (t < MTILE ? (int64_t)mi.P : (int64_t)mi.Q) * MTILE + (t & (MTILE - 1));
        const int64_t slot = mi.slot0 + (rw < mi.ne ? rw : (int64_t)mi.ne - 1);
        ms.thrA[t] = a.thrA[slot];
        ms.thrB[t] = a.thrB[slot];
    }
    const int sub = wm * 2 + (wn >> 1);                     // this wave's tile pair
    const bool active = (sub == 0 ? mi.blk[0] : sub == 1 ? mi.blk[1] : sub == 2 ? mi.blk[2] : mi.blk[3]) >= 0;
    MacroAcc acc;
#pragma unroll 1
    for (int st = 0; st < nst; ++st) {
        vm_wait<0>();                                       // this wave's part of stage st has landed
        lds_barrier();                                      // ... everyone's; stage st - 1 fully read
        if (st + 1 < nst) macro_issue(feed, st_lds + (uint32_t)(((st + 1) & 1) * MSTAGE), w, (uint32_t)(st + 1) * GROW);
        if (active) {
            if (st == 0) macro_mfma<PREC, true>(stages, acc, wm, wn);
            else macro_mfma<PREC, false>(stages + (st & 1) * MSTAGE, acc, wm, wn);
        }
    }
    const int I = 2 * mi.P + wm, J = 2 * mi.Q + (wn >> 1);
    if (active) {
        const int li = lane & 31, lg = lane >> 5;
        const bool full = I != J && (int64_t)(I + 1) * TILE <= mi.ne && (int64_t)(J + 1) * TILE <= mi.ne;
        int colc[2] = {0, 0};
        if (full) {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    colc[cb] += macro_block<true>(ms, sub, I, J, mi.ne, acc.c[rb][cb], rb, cb, wm, wn);
        } else {
#pragma unroll
            for (int rb = 0; rb < 4; ++rb)
#pragma unroll
                for (int cb = 0; cb < 2; ++cb)
                    colc[cb] += macro_block<false>(ms, sub, I, J, mi.ne, acc.c[rb][cb], rb, cb, wm, wn);
        }
#pragma unroll
        for (int cb = 0; cb < 2; ++cb) ms.colcnt[sub][lg][(wn & 1) * 64 + cb * 32 + li] = (uint8_t)colc[cb];
    }
    lds_barrier();
    // output: thread t serves row (and column) t % 128 of tile pair t / 128
    const int t = threadIdx.x;
    const int os = t >> 7, r = t & (TILE - 1);
    const int64_t blk = os == 0 ? mi.blk[0] : os == 1 ? mi.blk[1] : os == 2 ? mi.blk[2] : mi.blk[3];
    if (blk < 0) return;
    TilePos tl;
    tl.e = mi.e;
    tl.I = 2 * mi.P + (os >> 1);
    tl.J = 2 * mi.Q + (os & 1);
    tl.ne = mi.ne;
    tl.slot0 = mi.slot0;
    tl.blk = blk;
    const u32x4 wv = *(const u32x4 *)(ms.words[os] + 4 * r);
    *(u32x4 *)(a.bitmask + (uint64_t)blk * TILE_WORDS + 4 * r) = wv;
    const int64_t gr = (int64_t)tl.I * TILE + r;
    const int rc = __popc(wv.x) + __popc(wv.y) + __popc(wv.z) + __popc(wv.w);
    if (gr < tl.ne && rc) atomicAdd(&a.count[tl.slot0 + gr], rc);
    const int64_t gc = (int64_t)tl.J * TILE + r;
    const int cc = (int)ms.colcnt[os][0][r] + ms.colcnt[os][1][r];
    if (gc < tl.ne && cc) atomicAdd(&a.count[tl.slot0 + gc], cc);
    const u32x4 bw = *(const u32x4 *)(ms.bwords[os] + 4 * r);
    if (bw.x | bw.y | bw.z | bw.w) band_append(a, tl, r, bw, 0);
}

__global__ void k_build_macro_items(TileTable mt, TileTable tt, MacroItem *items, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    items[i] = macro_decode(mt, tt, i);
}

// ------------------------------------------------------------------- k-NN
// k-th nearest-neighbour squared distances over the whole cloud (the
// eps-selection module of the CIFAR-10 use case plots their distribution).
// Same Gram tiles and certified error bound as the eps tiles, over the
// T x T grid of 128-row blocks (on a cloud with cells, over the column
// blocks k_knn_lists leaves each row block): with hU_s >= |x_s|^2/2 + e_s and
// hL_s <= |x_s|^2/2 - e_s (the packing thresholds at eps = 0),
//   L_ij = 2 (hL_i + hL_j - g) <= D_ij <= U_ij = 2 (hU_i + hU_j - g),
// each evaluated in FP32 with a relative margin 2^-22 (|S| + |g|) that covers
// its two roundings.  Pass 1: T_i = k-th smallest U_ij (j != i) >= the true
// k-th smallest D.  Pass 2: every j with L_ij <= T_i is a candidate; that
// set holds every j with D_ij <= the k-th smallest D, so the k-th smallest
// canonical FP64 D over the candidates (k_knn_final) is the exact answer.
// mode 1 (the largest D, for the eccentricity lens) runs the same passes on
// negated values: -L in pass 1 (its smallest is -max L), -U in pass 2, -D
// in the final step, k = 1.
//
// A workgroup owns row block I and a chunk of its column blocks.  After each
// tile's products the bounds go to LDS (the stage buffers, free by then),
// row r at rotation r so the row scans below are free of bank conflicts;
// thread t then scans row t % 128, columns 32 (t / 128) .. + 31.
__device__ __forceinline__ int knn_off(int r, int c) { return r * TILE + ((c + r) & (TILE - 1)); }

// b: the KM smallest values seen, ascending; insert u (dropping the largest).
template <int KM>
__device__ __forceinline__ void topk_insert(float (&b)[KM], float u) {
#pragma unroll
    for (int q = KM - 1; q > 0; --q) b[q] = fminf(b[q], fmaxf(b[q - 1], u));
    b[0] = fminf(b[0], u);
}

// KM: the length of pass 1's sorted lists (8 when k <= 8: eight fewer
// registers, so that two workgroups fit on a CU where the precision allows).
template <int PREC, int PASS, int KM>
__global__ void __launch_bounds__(NTG, ((PASS == 2 || KM <= 8) && Cfg<PREC>::PANELS == 1) ? 2 : 1)
k_knn(KnnArgs a) {
    __shared__ __attribute__((aligned(1024))) char stages[2 * GSTAGE];   // also the bound tile
    __shared__ float hI[TILE], hJ[TILE];
    float *U = (float *)stages;
    const int w = __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    const int wm = w >> 2, wn = w & 3;
    const int64_t bl = block_linear();
    if (bl >= (int64_t)a.T * a.C) return;                  // a padding block of the 2-D grid
    const int I = (int)(bl / a.C), ch = (int)(bl % a.C);
    // the column blocks of row block I: all of them, or its list (screened
    // by the cloud's cells); chunk ch of C takes an even share
    const int nJ = a.jlist ? a.jcount[I] : a.T;
    const int J0 = (int)((int64_t)ch * nJ / a.C), J1 = (int)((int64_t)(ch + 1) * nJ / a.C);
    const int32_t *jl = a.jlist ? a.jlist + (int64_t)I * a.T : nullptr;
    const int r = threadIdx.x & (TILE - 1), qtr = threadIdx.x >> 7;
    const int64_t grow = (int64_t)I * TILE + r;
    const bool rvalid = grow < a.n;
    const bool upper = (PASS == 1) != (a.mode == 1);       // which bound this pass needs
    const float sgn = a.mode == 1 ? -1.f : 1.f;
    const float *hsrc = upper ? a.hU : a.hL;
    const uint32_t stride = (uint32_t)panel_row_stride(PREC, a.t.dp);
    const int nst = (int)(panel_row_bytes(PREC, a.t.dp) / GROW);
    const uint32_t st_lds = lds_addr(stages);
    float best[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) best[q] = __builtin_inff();
    const float thr_r = PASS == 2 ? a.thr[rvalid ? grow : a.n - 1] : 0.f;
    if (threadIdx.x < TILE) {
        const int64_t gi = (int64_t)I * TILE + threadIdx.x;
        hI[threadIdx.x] = hsrc[gi < a.n ? gi : a.n - 1];
    }
#pragma unroll 1
    for (int jp = J0; jp < J1; ++jp) {
        const int J = jl ? jl[jp] : jp;
        TilePos tl;
        tl.e = 0;
        tl.I = I;
        tl.J = J;
        tl.ne = a.n;
        tl.slot0 = 0;
        tl.blk = 0;
        GridFeed feed;
        grid_setup(a.t, tl, w, lane, stride, feed);
        grid_issue(feed, st_lds, w, 0);
        if (threadIdx.x < TILE) {
            const int64_t gj = (int64_t)J * TILE + threadIdx.x;
            hJ[threadIdx.x] = hsrc[gj < a.n ? gj : a.n - 1];
        }
        Acc<PREC> acc;
        GridOps ops;
#pragma unroll 1
        for (int st = 0; st < nst; ++st) {
            vm_wait<0>();
            lds_barrier();
            if (st + 1 < nst) grid_issue(feed, st_lds + (uint32_t)(((st + 1) & 1) * GSTAGE), w, (uint32_t)(st + 1) * GROW);
            grid_read<PREC>(stages + (st & 1) * GSTAGE, ops, wm, wn);
            if (st == 0) grid_mfma<PREC, true>(ops, acc);
            else grid_mfma<PREC, false>(ops, acc);
        }
        if constexpr (Cfg<PREC>::PANELS == 2) {
#pragma unroll
            for (int bm = 0; bm < 2; ++bm) acc.c[bm] = acc.c[bm] + acc.x[bm];
        }
        lds_barrier();                                      // every wave is done with the stages
        {
            const int li = lane_id_here();
            const int col = wn * 32 + (li & 31);
            const float hj = hJ[col];
#pragma unroll
            for (int bm = 0; bm < 2; ++bm)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const int row = wm * 64 + bm * 32 + 8 * (v >> 2) + 4 * (li >> 5) + (v & 3);
                    const float g = acc.c[bm][v];
                    const float S = hI[row] + hj;
                    const float m = 0x1.0p-22f * (fabsf(S) + fabsf(g));
                    U[knn_off(row, col)] = sgn * (upper ? 2.f * ((S - g) + m) : 2.f * ((S - g) - m));
                }
        }
        lds_barrier();
        if (rvalid) {
#pragma unroll 4
            for (int i = 0; i < 32; ++i) {
                const int col = 32 * qtr + i;
                const int64_t gcol = (int64_t)J * TILE + col;
                if (gcol >= a.n || gcol == grow) continue;
                const float u = U[knn_off(r, col)];
                if constexpr (PASS == 1) {
                    if (u < best[KM - 1]) topk_insert(best, u);
                } else {
                    if (u <= thr_r) {
                        const int slot = atomicAdd(&a.ccnt[grow], 1);
                        if (slot < a.cmax) a.cand[grow * a.cmax + slot] = (int32_t)gcol;
                    }
                }
            }
        }
        lds_barrier();                                      // the bound tile is read; stages free
    }
    if constexpr (PASS == 1) {
        const int64_t rows = (int64_t)a.T * TILE;
        float *dst = a.part + (((int64_t)ch * rows + grow) * 4 + qtr) * KNN_KMAX;
#pragma unroll
        for (int q = 0; q < KNN_KMAX; ++q) dst[q] = q < KM ? best[q < KM ? q : KM - 1] : __builtin_inff();
    }
}

// T_i = the k-th smallest of row i's partial lists (chunks x quarters).
__global__ void k_knn_merge(const float *part, int32_t C, int32_t T, int64_t n, int32_t k, float *thr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float best[KNN_KMAX];
#pragma unroll
    for (int q = 0; q < KNN_KMAX; ++q) best[q] = __builtin_inff();
    const int64_t rows = (int64_t)T * TILE;
    for (int c = 0; c < C; ++c)
        for (int qt = 0; qt < 4; ++qt) {
            const float *src = part + (((int64_t)c * rows + i) * 4 + qt) * KNN_KMAX;
            for (int q = 0; q < KNN_KMAX; ++q) {
                const float u = src[q];
                if (u < best[KNN_KMAX - 1]) topk_insert(best, u);
            }
        }
    float kth = best[0];
#pragma unroll
    for (int q = 1; q < KNN_KMAX; ++q) kth = q == k - 1 ? best[q] : kth;
    thr[i] = kth;
}

// The exact answer: the k-th smallest canonical FP64 D (x_j - y_j in FP64,
// fma in index order) over row i's candidates.  Rows and candidates are
// slots; perm (null: the identity) gives each slot's point, and the result
// goes to the point's entry.  One wave per row.  Each candidate's D is first
// summed in any order (lanes over the coordinates, a tree across the wave,
// the candidate's row read whole at once): that sum a lies within e = cf a / 2
// of the canonical chain (the bound of k_recheck, whose cf has a factor 2
// of margin).  With A the k-th smallest a, U = A (1 + cf) and L = A (1 - cf):
// a candidate with a (1 - cf) > U is not among the k smallest (k candidates
// lie at or below U), and one with a (1 + cf) < L is surely among the first
// k - 1 (fewer than k lie below A (1 - cf / 2)), so the answer is the
// (k - below)-th smallest canonical D of the rest, which alone take the
// canonical chain: one per row unless values nearly tie.  Signed values
// (-a, -D) in mode 1, with the same rules on |v|.
constexpr int KF_RG = 4;                 // candidates summed together (their row loads in flight at once)

template <int KM>
__device__ __forceinline__ void topk_insert_d(double (&b)[KM], double u) {
#pragma unroll
    for (int q = KM - 1; q > 0; --q) b[q] = fmin(b[q], fmax(b[q - 1], u));
    b[0] = fmin(b[0], u);
}

template <int KM>
__device__ __forceinline__ double pick_d(const double (&b)[KM], int k) {
    double v = b[0];                                         // b ascending: b[k - 1] = max(b[0 .. k - 1])
#pragma unroll
    for (int q = 1; q < KM; ++q) v = fmax(v, q < k ? b[q] : b[0]);
    return v;
}

// the wave's sums of (x_j - y_j)^2 for KF_RG rows y (every lane gets them)
__device__ __forceinline__ void knn_wave_sums(const float *x, const float *const (&y)[KF_RG], int32_t d, int lane,
                                              double (&s)[KF_RG]) {
#pragma unroll
    for (int i = 0; i < KF_RG; ++i) s[i] = 0.0;
    for (int j0 = 0; j0 < d; j0 += 4 * WAVE) {
        float xv[4], yv[KF_RG][4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int j = j0 + q * WAVE + lane;
            const int jj = j < d ? j : d - 1;                // in bounds; the term is dropped below
            xv[q] = x[jj];
#pragma unroll
            for (int i = 0; i < KF_RG; ++i) yv[i][q] = y[i][jj];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const bool live = j0 + q * WAVE + lane < d;
#pragma unroll
            for (int i = 0; i < KF_RG; ++i) {
                const double t = live ? (double)xv[q] - (double)yv[i][q] : 0.0;
                s[i] = __builtin_fma(t, t, s[i]);
            }
        }
    }
#pragma unroll
    for (int o = WAVE / 2; o > 0; o >>= 1)
#pragma unroll
        for (int i = 0; i < KF_RG; ++i) s[i] += __shfl_xor(s[i], o, WAVE);
}

template <int KM>
__global__ void __launch_bounds__(256) k_knn_final(const float *X, int32_t d, int64_t n, int32_t k, const int32_t *cand,
                                                   const int32_t *ccnt, int32_t cmax, int32_t mode,
                                                   const uint32_t *perm, double *out) {
    const int64_t i = block_linear() * 4 + __builtin_amdgcn_readfirstlane(threadIdx.x / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    if (i >= n) return;                                      // the whole wave leaves together
    const int cnt = ccnt[i] < cmax ? ccnt[i] : cmax;
    const int64_t pi = perm ? (int64_t)perm[i] : i;
    const float *x = X + pi * d;
    const int32_t *ci = cand + i * (int64_t)cmax;
    const double u = 0x1.0p-53;
    const double gd = (d + 4) * u / (1.0 - (d + 4) * u);
    const double cf = 4.0 * gd / (1.0 - gd);
    const double sg = mode == 1 ? -1.0 : 1.0;
    auto rows = [&](int c0, const float *(&y)[KF_RG]) {
#pragma unroll
        for (int q = 0; q < KF_RG; ++q) {
            const int c = c0 + q < cnt ? c0 + q : cnt - 1;   // past the end: the last candidate again
            const int64_t sc = ci[c];
            y[q] = X + (perm ? (int64_t)perm[sc] : sc) * d;
        }
    };
    // the k smallest signed sums; lane c keeps candidate c's
    double bv[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) bv[q] = __builtin_inf();
    double mine = 0.0;
    for (int c0 = 0; c0 < cnt; c0 += KF_RG) {
        const float *y[KF_RG];
        rows(c0, y);
        double sm[KF_RG];
        knn_wave_sums(x, y, d, lane, sm);
#pragma unroll
        for (int q = 0; q < KF_RG; ++q) {
            if (c0 + q < cnt) {
                topk_insert_d<KM>(bv, sg * sm[q]);
                if (lane == c0 + q) mine = sg * sm[q];
            }
        }
    }
    const double A = pick_d<KM>(bv, k);
    const double U = A + cf * fabs(A), L = A - cf * fabs(A);
    int below = 0;
    double best[KM];
#pragma unroll
    for (int q = 0; q < KM; ++q) best[q] = __builtin_inf();
    for (int c0 = 0; c0 < cnt; c0 += KF_RG) {
        double v[KF_RG];
        if (c0 < WAVE) {                                     // kept from the first sweep
#pragma unroll
            for (int q = 0; q < KF_RG; ++q) v[q] = __shfl(mine, c0 + q, WAVE);
        } else {                                             // summed again
            const float *y[KF_RG];
            rows(c0, y);
            double sm[KF_RG];
            knn_wave_sums(x, y, d, lane, sm);
#pragma unroll
            for (int q = 0; q < KF_RG; ++q) v[q] = sg * sm[q];
        }
#pragma unroll
        for (int q = 0; q < KF_RG; ++q) {
            if (c0 + q >= cnt) break;
            const double e = cf * fabs(v[q]);
            if (v[q] + e < L) {
                ++below;
            } else if (v[q] - e <= U) {                      // the canonical chain decides
                const int64_t sc = ci[c0 + q];
                const float *y = X + (perm ? (int64_t)perm[sc] : sc) * d;
                double D = 0.0;
                if (lane == 0)
                    for (int32_t j = 0; j < d; ++j) {
                        const double t = (double)x[j] - (double)y[j];
                        D = __builtin_fma(t, t, D);
                    }
                topk_insert_d<KM>(best, sg * __shfl(D, 0, WAVE));
            }
        }
    }
    const double kth = pick_d<KM>(best, k - below);
    if (lane == 0) out[pi] = sg * kth;
}

// Column-block lists of the k-NN passes over slots in cell order: jlist[I *
// T + p] (p < jcount[I]) = the column blocks J whose cells (cmask) meet
// those row block I may need.  Any set of columns gives pass 1 a valid
// bound (an upper bound of the k-th smallest, a lower bound of the
// largest), and pass 2 must keep every block that may hold a point a row
// of I needs; gap and far are the lower and upper bounds of the distance
// between two cells' points (nall x nall; far +inf where the outlier cell
// takes part, gap not positive where it says nothing), and the canonical
// FP64 distance lies within a factor 1 -+ (d + 8) 2^-52 (shrink, 2 - shrink)
// of the exact one.
//   mode 0 (k-th smallest), pass 1: the cells of I itself.  Pass 2: every
// cell whose ball may lie within sqrt(tau) of a cell of I, tau the largest
// of its rows' pass-1 bounds: a block farther than that holds no point
// within any row's k-th smallest bound.
//   mode 1 (the largest), pass 1: the cells of the farthest landmarks of
// I's rows (fmask; a row's farthest point usually lies there, so the bound
// loses little), or without fmask, for each cell a of I every cell whose
// far bound from a reaches the largest gap from a (the others cannot hold
// a row's farthest point).  Pass 2: every cell
// that may reach sqrt(tau) from a cell of I, tau the smallest of its rows'
// pass-1 bounds: a block nearer than that holds no point at the largest
// distance of any row.
// Pass 1 also takes blocks I - 1 .. I + 1.  thr is in panel units
// (inv_scale2 converts, with a margin of 2^-20); a row without a finite
// bound, or a cell of I that the tables say nothing about, keeps every
// block.  One wave per row block.
__global__ void __launch_bounds__(256) k_knn_lists(int32_t T, int64_t n, int32_t mode,
                                                   const unsigned long long *__restrict__ cmask,
                                                   const unsigned long long *__restrict__ fmask,
                                                   const double *__restrict__ gap, const double *__restrict__ far,
                                                   int32_t nall, const float *__restrict__ thr, double inv_scale2,
                                                   double shrink, int32_t *__restrict__ jlist,
                                                   int32_t *__restrict__ jcount) {
    const int64_t I = block_linear() * 4 + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (I >= T) return;                                      // the whole wave leaves together
    const unsigned long long cI = cmask[I];
    unsigned long long nm = cI;
    if (!thr && mode == 1 && fmask) {
        nm = fmask[I];
    } else if (!thr && mode == 1) {
        bool keep = false;
        unsigned long long m = cI;
        while (m) {
            const int ca = __ffsll((long long)m) - 1;
            m &= m - 1;
            double g = lane < nall && lane != ca ? gap[(int64_t)ca * nall + lane] : -1.0;
            for (int o = WAVE / 2; o > 0; o >>= 1) g = fmax(g, __shfl_xor(g, o, WAVE));
            // every cell that may hold a point farther than the farthest
            // cell's nearest point (all when the gaps say nothing)
            if (lane < nall && !(g > 0.0 && far[(int64_t)ca * nall + lane] < g)) keep = true;
        }
        nm = __ballot(keep);
    } else if (thr) {
        float t = -__builtin_inff();
        for (int r = lane; r < TILE; r += WAVE) {
            const int64_t row = I * TILE + r;
            if (row < n) t = fmaxf(t, thr[row]);
        }
        for (int o = WAVE / 2; o > 0; o >>= 1) t = fmaxf(t, __shfl_xor(t, o, WAVE));
        const double tau = mode == 1 ? -(double)t * inv_scale2 * (1.0 - 0x1.0p-20)
                                     : (double)t * inv_scale2 * (1.0 + 0x1.0p-20);
        if (!(t < __builtin_inff()) || (mode == 1 && !(tau > 0.0))) {
            nm = ~0ull;
        } else {
            const double grow = 2.0 - shrink;
            bool keep = false;
            if (lane < nall) {
                unsigned long long m = cI;
                while (m) {
                    const int ca = __ffsll((long long)m) - 1;
                    m &= m - 1;
                    if (mode == 1) {
                        const double f = far[(int64_t)ca * nall + lane];
                        if (!(f * f * grow < tau)) keep = true;
                    } else {
                        const double g = gap[(int64_t)ca * nall + lane];
                        if (!(ca != lane && g > 0.0 && g * g * shrink > tau)) keep = true;
                    }
                }
            }
            nm = __ballot(keep);
        }
    }
    int cnt = 0;
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (WAVE - lane));
    for (int J0 = 0; J0 < T; J0 += WAVE) {
        const int J = J0 + lane;
        // pass 1 also takes the neighbouring blocks I - 1 .. I + 1: with
        // them every row sees at least 128 others, so each pass-1 bound is
        // finite even where a row's own cells hold fewer than k points
        const bool keep = J < T && ((nm & cmask[J]) != 0 || (!thr && J >= I - 1 && J <= I + 1));
        const uint64_t b = __ballot(keep);
        if (keep) jlist[I * T + cnt + __popcll(b & below)] = J;
        cnt += __popcll(b);
    }
    if (lane == 0) jcount[I] = cnt;
}

// Band records from the band masks of the tile pair form: one wave per
// (level, tile pair).  Word w * 64 + l of the pair's mask block belongs to
// lane l of wave w of its workgroup (wave (wm, wn) = (w / 4, w % 4)): column
// wn * 32 + l % 32; bit 31 - v for value v of accumulator block 0, bit
// 15 - v for block 1, on the rows of the accumulator layout.  A tile pair
// with any band bit reserves its records with one atomic on its segment
// (segment (t / 32) mod nseg for tile pair t: 32 consecutive tile pairs
// share one, so their records and rows stay together for the recheck) and
// every lane writes its own; past band_cap they are only counted.
__global__ void __launch_bounds__(256) k_band_collect(const TileItem *__restrict__ items, int64_t n_items,
                                                      const uint32_t *__restrict__ bandmask, int32_t n_levels,
                                                      uint64_t level_words, BandPair *__restrict__ band,
                                                      unsigned long long *__restrict__ band_n, int64_t band_cap,
                                                      int32_t nseg) {
    const int64_t wv = block_linear() * 4 + threadIdx.x / WAVE;
    const int lane = threadIdx.x & (WAVE - 1);
    if (wv >= n_items * n_levels) return;                    // the whole wave leaves together
    const int lv = (int)(wv / n_items);
    const int64_t t = wv - (int64_t)lv * n_items;
    const TileItem it = items[t];
    const uint32_t *mb = bandmask + (uint64_t)lv * level_words + (uint64_t)it.blk * TILE_WORDS + lane;
    uint32_t m[8];
    int n = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        m[w] = mb[w * WAVE];
        n += __popc(m[w]);
    }
    if (__ballot(n != 0) == 0) return;                      // uniform: most tile pairs have no band pair
    int incl = n;                                            // inclusive prefix sum over the lanes
    for (int o = 1; o < WAVE; o <<= 1) {
        const int y = __shfl_up(incl, (unsigned)o, WAVE);
        if (lane >= o) incl += y;
    }
    const int total = __shfl(incl, WAVE - 1, WAVE);
    const int seg = (int)((t >> 5) % nseg);
    unsigned long long b = 0;
    if (lane == 0) b = atomicAdd(&band_n[seg], (unsigned long long)total);
    const uint32_t blo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t bhi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    int64_t idx = (int64_t)(((uint64_t)bhi << 32) | blo) + (incl - n);
    const int li = lane & 31, lg = lane >> 5;
#pragma unroll
    for (int w = 0; w < 8; ++w) {
        const int wm = w >> 2, wn = w & 3, cl = wn * 32 + li;
        uint32_t mm = m[w];
        while (mm) {
            const int k = __ffs(mm) - 1;
            mm &= mm - 1;
            const int bm = k >= 16 ? 0 : 1, v = 15 - (k & 15);
            const int rl = wm * 64 + bm * 32 + 4 * lg + 8 * (v >> 2) + (v & 3);
            if (idx < band_cap) {
                BandPair bp;
                bp.si = (int32_t)(it.slot0 + (int64_t)it.I * TILE + rl);
                bp.sj = (int32_t)(it.slot0 + (int64_t)it.J * TILE + cl);
                bp.bit = (((uint64_t)it.blk * TILE_WORDS + (uint64_t)(rl * 4 + wn)) * 32u + (uint64_t)li) |
                         ((uint64_t)lv << BAND_LEVEL_SHIFT);
                band[(int64_t)seg * band_cap + idx] = bp;
            }
            ++idx;
        }
    }
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
    const dim3 grid = grid_2d(8 * ((a.tt.n_items + 7) / 8));
    if (a.n_levels < 1 || a.n_levels > MAX_LEVELS || (a.debug_g && a.n_levels != 1)) return hipErrorInvalidValue;
    if (a.debug_g) k_tiles<PREC, true, 1><<<grid, dim3(NTG), 0, s>>>(a);
    else if (a.n_levels == 1) k_tiles<PREC, false, 1><<<grid, dim3(NTG), 0, s>>>(a);
    else k_tiles<PREC, false, MAX_LEVELS><<<grid, dim3(NTG), 0, s>>>(a);
    return hipGetLastError();
}

template <int PREC>
hipError_t launch_macro_t(const TileArgs &a, hipStream_t s) {
    if (a.n_mitems <= 0) return hipSuccess;
    if (a.n_levels != 1 || a.debug_g || !a.mitems) return hipErrorInvalidValue;
    // the stage offsets of a side's 256 rows are 32-bit
    if ((uint64_t)panel_row_stride(PREC, a.dp) * MTILE >= (1ull << 32)) return hipErrorInvalidValue;
    k_tiles_macro<PREC><<<grid_2d(8 * ((a.n_mitems + 7) / 8)), dim3(NTG), 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_tiles_macro(int prec, const TileArgs &a, hipStream_t s) {
    switch (prec) {
    case P_BF16: return launch_macro_t<P_BF16>(a, s);
    case P_FP16: return launch_macro_t<P_FP16>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_build_macro_items(const TileTable &mt, const TileTable &tt, MacroItem *items, int64_t n,
                                    hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_build_macro_items<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(mt, tt, items, n);
    return hipGetLastError();
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

template <int PREC>
hipError_t launch_knn_t(int pass, const KnnArgs &a, hipStream_t s) {
    const dim3 G = grid_2d((int64_t)a.T * a.C);
    if (pass == 1 && a.k <= 8) k_knn<PREC, 1, 8><<<G, dim3(NTG), 0, s>>>(a);
    else if (pass == 1) k_knn<PREC, 1, KNN_KMAX><<<G, dim3(NTG), 0, s>>>(a);
    else k_knn<PREC, 2, KNN_KMAX><<<G, dim3(NTG), 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_knn_pass(int prec, int pass, const KnnArgs &a, hipStream_t s) {
    if (a.n < 2 || a.T < 1 || a.C < 1 || (pass != 1 && pass != 2)) return hipErrorInvalidValue;
    switch (prec) {
    case P_FP32: return launch_knn_t<P_FP32>(pass, a, s);
    case P_BF16: return launch_knn_t<P_BF16>(pass, a, s);
    case P_BF16X3: return launch_knn_t<P_BF16X3>(pass, a, s);
    case P_FP16: return launch_knn_t<P_FP16>(pass, a, s);
    case P_FP16X3: return launch_knn_t<P_FP16X3>(pass, a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_knn_merge(const float *part, int32_t C, int32_t T, int64_t n, int32_t k, float *thr,
                            hipStream_t s) {
    k_knn_merge<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(part, C, T, n, k, thr);
    return hipGetLastError();
}

hipError_t launch_knn_final(const float *X, int32_t d, int64_t n, int32_t k, const int32_t *cand,
                            const int32_t *ccnt, int32_t cmax, int32_t mode, const uint32_t *perm, double *out,
                            hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (k <= 8)
        k_knn_final<8><<<grid_2d((n + 3) / 4), dim3(256), 0, s>>>(X, d, n, k, cand, ccnt, cmax, mode, perm, out);
    else
        k_knn_final<KNN_KMAX><<<grid_2d((n + 3) / 4), dim3(256), 0, s>>>(X, d, n, k, cand, ccnt, cmax, mode, perm,
                                                                          out);
    return hipGetLastError();
}

hipError_t launch_knn_lists(int32_t T, int64_t n, int32_t mode, const unsigned long long *cmask,
                            const unsigned long long *fmask, const double *gap, const double *far, int32_t nall,
                            const float *thr, double inv_scale2, double shrink, int32_t *jlist, int32_t *jcount,
                            hipStream_t s) {
    if (T <= 0) return hipSuccess;
    if (nall < 1 || nall > CELL_MAX || (mode != 0 && mode != 1)) return hipErrorInvalidValue;
    k_knn_lists<<<grid_2d(((int64_t)T + 3) / 4), dim3(256), 0, s>>>(T, n, mode, cmask, fmask, gap, far, nall, thr,
                                                                      inv_scale2, shrink, jlist, jcount);
    return hipGetLastError();
}

hipError_t launch_band_collect(const TileTable &tt, const uint32_t *bandmask, int32_t n_levels, uint64_t level_words,
                               BandPair *band, unsigned long long *band_n, int64_t band_cap, int32_t nseg,
                               hipStream_t s) {
    if (tt.n_items <= 0) return hipSuccess;
    if (n_levels < 1 || n_levels > MAX_LEVELS || nseg < 1) return hipErrorInvalidValue;
    const int64_t waves = tt.n_items * n_levels;
    k_band_collect<<<grid_2d((waves + 3) / 4), dim3(256), 0, s>>>(tt.items, tt.n_items, bandmask, n_levels,
                                                                   level_words, band, band_n, band_cap, nseg);
    return hipGetLastError();
}

hipError_t launch_build_items(const TileTable &tt, TileItem *items, hipStream_t s) {
    if (tt.n_items <= 0) return hipSuccess;
    k_build_items<<<dim3((unsigned)((tt.n_items + 255) / 256)), dim3(256), 0, s>>>(tt, items);
    return hipGetLastError();
}

}  // namespace mgpu
