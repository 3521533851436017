// internal.h -- declarations shared by the host runtime and the HIP kernels of
// libmapper_gpu.  Not part of the public ABI (include/mapper_gpu.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>
#include <cstddef>
#include <stdexcept>
#include <vector>

namespace mgpu {

// ---------------------------------------------------------------- tiling
// Distance tiles are TILE x TILE blocks of one cover element's members.
constexpr int TILE = 128;
constexpr int MAX_LEVELS = 4;        // eps values one tile pass can serve
constexpr int TILE_WORDS = TILE * TILE / 32;      // uint32 words of one bitmask block
constexpr int WAVE = 64;

enum Prec : int { P_FP32 = 0, P_BF16 = 1, P_BF16X3 = 2, P_FP16 = 3, P_FP16X3 = 4 };

// One dimension of a dispatch covers at most 2^32 - 1 work-items, so the
// launches with a workgroup (or a wave) per tile pair -- millions of them --
// use a 2-D grid of at most GRID_ROW workgroups per row.  Rows are as short
// as the row count allows, rounded up to a multiple of 8: fewer than 8
// padding workgroups per row (they exit at once), and the hardware's
// round-robin of workgroups over the 8 XCDs follows the linear index
// (block_linear) that those kernels map to their items.
constexpr int64_t GRID_ROW = 1 << 16;
inline dim3 grid_2d(int64_t blocks) {
    if (blocks <= GRID_ROW) return dim3((unsigned)blocks, 1u);
    const int64_t gy = (blocks + GRID_ROW - 1) / GRID_ROW;
    const int64_t gx = 8 * (((blocks + gy - 1) / gy + 7) / 8);
    return dim3((unsigned)gx, (unsigned)gy);
}
__device__ __forceinline__ int64_t block_linear() { return (int64_t)blockIdx.y * gridDim.x + blockIdx.x; }

inline bool prec_is_split(int p) { return p == P_BF16X3 || p == P_FP16X3; }
inline bool prec_is_16bit(int p) { return p != P_FP32; }
inline bool prec_is_bf16(int p) { return p == P_BF16 || p == P_BF16X3; }

// Work table of the distance-tile launch.  Items are the tile pairs (I <= J)
// of all elements, grouped by element in the order `order` (largest first).
// Inside an element the tile pairs are visited in supertiles of S x S pairs
// (upper triangle only), supertile columns left to right, supertiles of a
// column top to bottom, and inside a supertile row blocks fastest.  Workgroups
// that run together on one XCD thus share a few row panels in its L2.  S is
// chosen per run (TileTable::super, supertile_size below).

// One tile pair, decoded (32 bytes: one scalar load per workgroup or wave).
struct __attribute__((aligned(32))) TileItem {
    int32_t e, I, J, ne;       // element, row block, column block, element size
    int64_t slot0, blk;        // first slot of the element, bitmask block
};

struct TileTable {
    const int64_t *item_off;   // [nord+1] first item of each ordered element
    const int32_t *order;      // [nord] element id of each ordered entry
    const int64_t *elem_off;   // [E+1] first slot of each element
    const int64_t *blk_off;    // [E] first bitmask block of each element
    const int64_t *colpre;     // per element: items before each supertile column (Ts+1)
    const int64_t *cp_off;     // [E] start of the element's colpre entries
    const struct TileItem *items;   // decoded items, built by launch_build_items
    int32_t nord;
    int32_t super;             // supertile size S
    int64_t n_items;
};

struct TilePos {
    int e, I, J;
    int64_t ne, slot0, blk;
};

// Item (global tile-pair index) -> element, row block I, column block J (I <= J)
// and the bitmask block that stores it, for blocks of `tr` rows (TILE for the
// tile pairs, MTILE for the macro tiles below).
__host__ __device__ __forceinline__ TilePos tile_decode_rows(const TileTable &t, int64_t item, int64_t tr) {
    int lo = 0, hi = t.nord;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (t.item_off[mid] <= item) lo = mid; else hi = mid;
    }
    TilePos r;
    r.e = t.order[lo];
    const int64_t p = item - t.item_off[lo];
    r.slot0 = t.elem_off[r.e];
    r.ne = t.elem_off[r.e + 1] - r.slot0;
    r.blk = t.blk_off[r.e] + p;
    const int64_t T = (r.ne + tr - 1) / tr;
    const int64_t S = t.super;
    const int64_t Ts = (T + S - 1) / S;
    const int64_t *cp = t.colpre + t.cp_off[r.e];
    int64_t a = 0, b = Ts;                         // largest SJ with cp[SJ] <= p
    while (b - a > 1) {
        const int64_t mid = (a + b) >> 1;
        if (cp[mid] <= p) a = mid; else b = mid;
    }
    const int64_t SJ = a;
    const int64_t q = p - cp[SJ];
    const int64_t cols = (T - SJ * S) < S ? (T - SJ * S) : S;
    const int64_t per = S * cols;
    if (q < SJ * per) {
        const int64_t SI = q / per, loc = q - SI * per;
        r.I = (int)(SI * S + loc % S);
        r.J = (int)(SJ * S + loc / S);
    } else {
        const int64_t loc = q - SJ * per;
        int64_t j = (int64_t)((sqrt(8.0 * (double)loc + 1.0) - 1.0) * 0.5);
        while ((j + 1) * (j + 2) / 2 <= loc) ++j;
        while (j * (j + 1) / 2 > loc) --j;
        r.I = (int)(SJ * S + (loc - j * (j + 1) / 2));
        r.J = (int)(SJ * S + j);
    }
    return r;
}

__host__ __device__ __forceinline__ TilePos tile_decode(const TileTable &t, int64_t item) {
    return tile_decode_rows(t, item, TILE);
}

// The decoded item from the table (one scalar load instead of the searches).
__device__ __forceinline__ TilePos tile_lookup(const TileTable &t, int64_t item) {
    const TileItem q = t.items[item];
    TilePos r;
    r.e = q.e;
    r.I = q.I;
    r.J = q.J;
    r.ne = q.ne;
    r.slot0 = q.slot0;
    r.blk = q.blk;
    return r;
}

// Inverse of tile_decode inside one element: the position p of tile pair
// (I, J), I <= J < T, in the element's order of supertiles of size S (cp = its
// colpre).
__host__ __device__ __forceinline__ int64_t tile_local_index(const int64_t *cp, int64_t T, int64_t S,
                                                             int64_t I, int64_t J) {
    const int64_t SI = I / S, SJ = J / S;
    const int64_t cols = (T - SJ * S) < S ? (T - SJ * S) : S;
    const int64_t per = S * cols;
    if (SI < SJ) return cp[SJ] + SI * per + (I % S) + S * (J % S);
    const int64_t i = I % S, j = J % S;
    return cp[SJ] + SJ * per + j * (j + 1) / 2 + i;
}

// Items before each supertile column of every element (host; T[e] = tile
// rows of element e, S = supertile size): the colpre table of tile_decode.
inline void build_supertile_columns(const std::vector<int64_t> &T, int64_t S, std::vector<int64_t> &colpre,
                                    std::vector<int64_t> &cp_off) {
    colpre.clear();
    for (size_t e = 0; e < T.size(); ++e) {
        const int64_t Ts = (T[e] + S - 1) / S;
        cp_off[e] = (int64_t)colpre.size();
        int64_t acc = 0;
        colpre.push_back(0);
        for (int64_t SJ = 0; SJ < Ts; ++SJ) {
            const int64_t cols = std::min<int64_t>(S, T[e] - SJ * S);
            acc += SJ * S * cols + cols * (cols + 1) / 2;
            colpre.push_back(acc);
        }
        if (acc != T[e] * (T[e] + 1) / 2) throw std::runtime_error("supertile table mismatch");
    }
    if (colpre.empty()) colpre.push_back(0);
}

// Macro tiles: pairs of 256-row blocks (P <= Q) of one element, each holding up
// to four tile pairs (2P + a, 2Q + b), a, b in {0, 1}, kept when
// 2P + a <= 2Q + b < T.  A macro table is a TileTable over blocks of MTILE
// rows (its own supertile columns, the same element order); the tile pairs
// keep their bitmask blocks in the tile table's order, so every consumer of
// the bitmask reads the same layout whichever form computed it.
constexpr int MTILE = 2 * TILE;

struct __attribute__((aligned(64))) MacroItem {
    int32_t e, P, Q, ne;       // element, macro row and column blocks, element size
    int64_t slot0;             // first slot of the element
    int64_t blk[4];            // bitmask block of tile pair (2P + a, 2Q + b) at [2a + b]; -1 if absent
    int64_t pad;
};

// Macro item `item` of macro table mt, with the bitmask blocks of its tile
// pairs from the tile table tt (both over the same elements).
__host__ __device__ inline MacroItem macro_decode(const TileTable &mt, const TileTable &tt, int64_t item) {
    const TilePos m = tile_decode_rows(mt, item, MTILE);
    MacroItem r;
    r.e = m.e;
    r.P = m.I;
    r.Q = m.J;
    r.ne = (int32_t)m.ne;
    r.slot0 = m.slot0;
    r.pad = 0;
    const int64_t T = (m.ne + TILE - 1) / TILE;
    const int64_t *cp = tt.colpre + tt.cp_off[m.e];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            const int64_t I = 2 * (int64_t)m.I + a, J = 2 * (int64_t)m.J + b;
            r.blk[2 * a + b] = (I < T && J < T && I <= J)
                                   ? tt.blk_off[m.e] + tile_local_index(cp, T, tt.super, I, J) : -1;
        }
    return r;
}

// One pair whose tile distance fell inside the certified band of eps^2.
struct BandPair {
    int32_t si, sj;            // slots (global member positions)
    uint64_t bit;              // bit index in the level's bitmask | level << BAND_LEVEL_SHIFT
};
constexpr int BAND_LEVEL_SHIFT = 56;
// The levels' eps^2 and strides, for the FP64 re-decision of band pairs.
struct Levels {
    double E[MAX_LEVELS];
    int64_t level_slots;       // count of level t at t * level_slots
    uint64_t level_words;      // bitmask of level t at t * level_words
};

// ---------------------------------------------------------------- launchers
// Every launcher enqueues on `s` and returns hipSuccess or the launch error.

// lens.hip
hipError_t launch_check_cloud(const float *X, int64_t count, uint32_t *flags_maxabs, hipStream_t s);
hipError_t launch_lens(const float *X, int64_t n, int32_t d, int kind, int32_t column,
                       const float *dir, const double *values, double *f, hipStream_t s);
hipError_t launch_range(const double *f, int64_t n, unsigned long long *keys2, hipStream_t s);
// keys[i] = order-preserving key of f[i], vals[i] = i (for a radix sort of the lens).
hipError_t launch_lens_keys(const double *f, int64_t n, uint64_t *keys, uint32_t *vals, hipStream_t s);
// out[i] = the lens value whose key is sorted[rank[i]] (zero as +0).
hipError_t launch_rank_values(const uint64_t *sorted, const int64_t *rank, int32_t m, double *out,
                              hipStream_t s);

// prims.hip
size_t scan_temp_bytes(int64_t n);
// out[0..n] = exclusive prefix sums of in[0..n) (out[n] = total), int64.
hipError_t launch_scan_i32(const int32_t *in, int64_t *out, int64_t n, void *temp, hipStream_t s);
hipError_t launch_scan_i64(const int64_t *in, int64_t *out, int64_t n, void *temp, hipStream_t s);
hipError_t launch_scan_u8(const uint8_t *in, int64_t *out, int64_t n, void *temp, hipStream_t s);
size_t sort_temp_bytes(int64_t n);
// Stable LSD radix sort of (key, value) by the low key_bits of key.  Uses the
// *_alt buffers as ping-pong space; returns in *result_in_alt whether the
// sorted data ended in the alt buffers.
hipError_t radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt,
                            uint32_t *vals_alt, int64_t n, int key_bits, void *temp,
                            bool *result_in_alt, hipStream_t s);
// out[i] = i.
hipError_t launch_iota_u32(uint32_t *out, int64_t n, hipStream_t s);
// *out = max(*out, max of in[0..n)), for in[i] >= 0.
hipError_t launch_max_i32(const int32_t *in, int64_t n, int32_t *out, hipStream_t s);
// out[v] = first index i in sorted keys[0..n) with keys[i] >= v, v in [0, nv].
hipError_t launch_lower_bounds(const uint64_t *keys, int64_t n, int64_t nv, int64_t *out,
                               hipStream_t s);

// bin.hip
hipError_t launch_member_count(const double *f0, const double *f1, int64_t n,
                               const double *lo0, const double *hc0, int32_t n0,
                               const double *lo1, const double *hc1, int32_t n1,
                               int32_t *range4, int32_t *count, unsigned long long *pair_sum,
                               hipStream_t s);
// keys = element id << key_bits | okey[point] (okey may be null: 0)
hipError_t launch_member_emit(const int32_t *range4, const int64_t *pos, int64_t n, int32_t n1,
                              int two_d, const uint16_t *okey, int key_bits, uint64_t *keys, uint32_t *vals,
                              hipStream_t s);
// Packed panel rows.  A row holds dp coordinates: FP32 values (4 bytes), one
// 16-bit value each (BF16, FP16), or for the hi/lo splits groups of 16 hi
// values followed by their 16 lo values (4 bytes per coordinate).  dp is d
// rounded up so that a row is a whole number of 64-byte slabs, at least four.
__host__ __device__ inline int panel_dp(int prec, int d) {
    if (prec == P_FP32) return d <= 64 ? 64 : 32 * ((d + 31) / 32);
    if (prec == P_BF16X3 || prec == P_FP16X3) return 64 * ((d + 63) / 64);
    return d <= 128 ? 128 : 64 * ((d + 63) / 64);
}
__host__ __device__ inline int64_t panel_row_bytes(int prec, int dp) {
    return (int64_t)dp * ((prec == P_BF16 || prec == P_FP16) ? 2 : 4);
}
// Distance between consecutive rows: the row bytes padded to an odd number of
// 128-byte lines, so that the same slab of many rows spreads over all L2
// channels (a power-of-two row stride would put it on a few of them).
__host__ __device__ inline int64_t panel_row_stride(int prec, int dp) {
    const int64_t b = panel_row_bytes(prec, dp);
    return ((b >> 7) & 1) ? b : b + 128;
}

// Supertile size of a tile launch, the same for every precision (the tile
// order is fixed before the precision is chosen).  For the hi/lo splits,
// which read twice the bytes of a single 16-bit product per pair, 24 x 24
// supertiles (24 row panels of at most 144 KB, about 3.4 MB, inside an XCD's
// 4 MB L2) were measured 2-3% faster than 8 x 8 at 1M x 256, while 32 x 32
// overflows the L2 and is slower; single products were within 1% from 4 x 4
// to 24 x 24.  Rows longer than 256 coordinates keep 8 x 8.
inline int supertile_size(int d) { return d <= 256 ? 24 : 8; }

struct PackArgs {
    const float *X; int32_t d; int32_t dp;
    const uint32_t *slot_point; int64_t n_slots;
    int prec;
    double scale;              // power of two applied to coordinates
    int32_t n_levels;          // eps values served by one tile pass (1 .. MAX_LEVELS)
    double E_scaled[MAX_LEVELS];   // eps_t^2 * scale^2
    void *panel;               // packed rows (panel_row_bytes each, panel_row_stride apart)
    float *thrA; float *thrB;  // in-threshold / out-threshold of each slot, level t at t * n_slots
    double *dbg_norm2;         // optional: |x_s|^2 (scaled)
    double *dbg_e;             // optional: e_s, the slot's share of the Gram error bound (scaled)
};
hipError_t launch_pack(const PackArgs &a, hipStream_t s);

// cells.hip: landmark cells of a cloud (at most CELL_MAX - 2 landmarks,
// staged whole in LDS: ncell * d <= CELL_LDS_FLOATS).  Cell ids fit a 64-bit
// mask: the landmarks 0 .. ncell - 1, the outlier cell ncell, and at run
// time ncell + 1 for outliers farther than eps from every landmark cell.
constexpr int CELL_MAX = 64;
constexpr int CELL_LDS_FLOATS = 16384;
// cell[i] = nearest landmark, or ncell (the outlier cell) past limit2[c]
// (squared distance); ncell + 1 < CELL_MAX.  landT: the landmarks
// transposed, d x CELL_MAX (zero past ncell); lnorm[c] = |l_c|^2 (FP32).
hipError_t launch_assign_cells(const float *X, int64_t n, int32_t d, const float *landT, const float *lnorm,
                               int32_t ncell, const float *limit2, uint8_t *cell, uint8_t *far, hipStream_t s);
// out[i] = squared distance from sample row i to its nearest other row.
hipError_t launch_sample_nn2(const float *sub, int32_t m, int32_t d, float *out, hipStream_t s);
// out[i] = items[i * n / m] with blk = i (an evenly strided sample of a tile
// list, each with its own bitmask block).
hipError_t launch_sample_items(const TileItem *items, int64_t n, int64_t m, TileItem *out, hipStream_t s);
// keys[i] >>= shift
hipError_t launch_shift_keys(uint64_t *keys, int64_t n, int shift, hipStream_t s);
// The margins of the cell balls' bounds assume d <= BALL_DMAX.
constexpr int BALL_DMAX = 2048;
// Per row block (nrb of them, numbered by rb_off): cmask = its rows' cells,
// nmask = the cells near any of them (near: the table of cells that eps may
// join, one 64-bit mask per cell).
// A point of cell `outlier` whose ogap (null: none) passes the eps test
// g^2 shrink > Eb counts as cell outlier + 1.
hipError_t launch_tile_cells(const uint32_t *slot_point, const int64_t *elem_off, const int64_t *rb_off,
                             int32_t n_elem, int64_t nrb, const uint8_t *cell, const float *ogap, int32_t outlier,
                             double shrink, double Eb, const unsigned long long *near, unsigned long long *cmask,
                             unsigned long long *nmask, hipStream_t s);
// gap[i] = a lower bound of the distance from point i of the outlier cell
// (id ncell) to every point of the landmark cells (landmarks land, radius
// bounds rad), rounded down to FP32; -1 for the points of landmark cells.
hipError_t launch_outlier_gap(const float *X, int64_t n, int32_t d, const float *land, int32_t ncell,
                              const double *rad, const uint8_t *cell, float *gap, hipStream_t s);
// keep[i] = 0 if no cell of tile pair i's column block is near a cell of its
// row block (diagonal pairs are kept).
hipError_t launch_screen(const TileItem *items, int64_t n, const int64_t *rb_off, const unsigned long long *cmask,
                         const unsigned long long *nmask, uint8_t *keep, hipStream_t s);
// r2[c] = max |x - land_c|^2 over the points of cell c (double bits; r2
// zeroed by the caller).
hipError_t launch_cell_radius(const float *X, int64_t n, int32_t d, const float *land, int32_t ncell,
                              const uint8_t *cell, unsigned long long *r2, hipStream_t s);
// out[pos[i]] = items[i] with blk = pos[i] for kept items; diag_blk and
// next_blk (the blocks of (I, I) and (I, I + 1) at rb_off[e] + I, -1 if
// screened out; next_blk preset to -1 by the caller); the in-element pairs
// of the kept tile pairs are added to pairs[0 .. PAIR_SLOTS - 1] (zeroed by
// the caller, who sums them).
constexpr int PAIR_SLOTS = 64;
hipError_t launch_compact_items(const TileItem *items, int64_t n, const uint8_t *keep, const int64_t *pos,
                                const int64_t *rb_off, TileItem *out, int64_t *diag_blk, int64_t *next_blk,
                                unsigned long long *pairs, hipStream_t s);

// tile.hip
struct TileArgs {
    TileTable tt;
    const void *panel; int32_t dp;
    const float *thrA; const float *thrB;
    uint32_t *bitmask; int32_t *count;
    // band pairs: nseg segments of band_cap entries; band_n[g] counts the pairs
    // of segment g (past band_cap they are counted but not stored)
    BandPair *band; unsigned long long *band_n; int64_t band_cap; int32_t nseg;
    // tile pair form: per level and tile pair, one band-mask word per lane of
    // each of its eight waves (TILE_WORDS words, the bitmask's block layout
    // in size); k_band_collect turns them into band records
    uint32_t *bandmask;
    // eps values served by the pass: thresholds, counts and bitmask of level t
    // at t * level_slots (thrA, thrB, count) and t * level_words (bitmask)
    int32_t n_levels; int64_t level_slots; uint64_t level_words;
    float *debug_g;            // non-null: write raw Gram values (debug, one element)
    int64_t debug_ld;
    const MacroItem *mitems;   // macro form: the decoded macro items (launch_build_macro_items)
    int64_t n_mitems;
};
hipError_t launch_tiles(int prec, const TileArgs &a, hipStream_t s);
// Band records of every tile pair of tt (its items) from the band masks the
// tile pair form left: n_levels levels level_words apart; segment = tile pair
// index mod nseg; band_n counts every pair, records past band_cap are not
// stored (band_n zeroed by the caller).
hipError_t launch_band_collect(const TileTable &tt, const uint32_t *bandmask, int32_t n_levels, uint64_t level_words,
                               BandPair *band, unsigned long long *band_n, int64_t band_cap, int32_t nseg,
                               hipStream_t s);
// The same bitmask, counts and band records as launch_tiles, computed by one
// workgroup per macro item (a.mitems); single 16-bit products (BF16, FP16),
// one eps value, no debug output.
hipError_t launch_tiles_macro(int prec, const TileArgs &a, hipStream_t s);
// items[i] = macro item i of the macro table mt over the tile table tt.
hipError_t launch_build_macro_items(const TileTable &mt, const TileTable &tt, MacroItem *items, int64_t n,
                                    hipStream_t s);
// k-th nearest-neighbour squared distances over the whole cloud (tile.hip).
constexpr int KNN_KMAX = 16;         // largest k

struct KnnArgs {
    TileArgs t;                        // panel, dp (the Gram tiles)
    int64_t n;                         // slots (the points, in the order of the packed panels)
    int32_t T, C;                      // row blocks; column-block chunks per row block
    const float *hU, *hL;              // per point, scaled (packing thresholds at eps = 0)
    float *part;                       // pass 1: per (chunk, row, quarter) the 16 smallest U
    const float *thr;                  // pass 2: T_i
    int32_t *cand, *ccnt;              // pass 2: candidates of row i at i * cmax, their count
    int32_t cmax;
    int32_t mode;                      // 0: k-th smallest D; 1: largest D (values negated)
    int32_t k;                         // the k of the k-th smallest (1 in mode 1)
    const int32_t *jlist, *jcount;     // null: every column block; else row block I's list at I * T, its length
};

hipError_t launch_knn_pass(int prec, int pass, const KnnArgs &a, hipStream_t s);
hipError_t launch_knn_merge(const float *part, int32_t C, int32_t T, int64_t n, int32_t k, float *thr,
                            hipStream_t s);
hipError_t launch_knn_final(const float *X, int32_t d, int64_t n, int32_t k, const int32_t *cand,
                            const int32_t *ccnt, int32_t cmax, int32_t mode, const uint32_t *perm, double *out,
                            hipStream_t s);
// Column-block lists of the screened k-NN passes (k_knn_lists): cmask per row
// block, gap and far the lower and upper bounds of the distance between two
// cells' points (nall x nall, device), thr null for pass 1; mode as k_knn;
// fmask (mode 1, pass 1; may be null) per row block the cells of its rows'
// farthest landmarks.
hipError_t launch_knn_lists(int32_t T, int64_t n, int32_t mode, const unsigned long long *cmask,
                            const unsigned long long *fmask, const double *gap, const double *far, int32_t nall,
                            const float *thr, double inv_scale2, double shrink, int32_t *jlist, int32_t *jcount,
                            hipStream_t s);
// f[i] = sqrt(f[i]) (correctly rounded FP64).
hipError_t launch_sqrt(double *f, int64_t n, hipStream_t s);
// items[i] = decoded tile pair i of the table (one thread per item).
hipError_t launch_build_items(const TileTable &tt, TileItem *items, hipStream_t s);
// band_n[g] = pairs in segment g (<= band_cap), nband their sum.
hipError_t launch_recheck(const BandPair *band, const unsigned long long *band_n, int32_t nseg,
                          int64_t band_cap, int64_t nband, const float *X, int32_t d,
                          const uint32_t *slot_point, const Levels &lv, uint32_t *bitmask, int32_t *count,
                          hipStream_t s);
hipError_t launch_row_norm2(const int32_t *rows, int64_t nr, const float *X, int32_t d,
                            double *out, hipStream_t s);
hipError_t launch_pair_d64(const int32_t *pa, const int32_t *pb, int64_t np, const float *X,
                           int32_t d, double *out, hipStream_t s);

// graph.hip
hipError_t launch_cc_init(int32_t *parent, int64_t n_slots, hipStream_t s);
// parent[i] = root of i for every slot (path compression).
hipError_t launch_cc_compress(int32_t *parent, int64_t n_slots, hipStream_t s);
hipError_t launch_cc_tiles(const TileTable &tt, const uint32_t *bitmask, const int32_t *count,
                           int32_t min_pts, int32_t *parent, hipStream_t s);
// diag_blk / next_blk: blocks of tile pairs (I, I) and (I, I + 1) of each
// element at rb_off[e] + I (-1: not computed), or null for the full table
// (tile_local_index).
hipError_t launch_cc_hook(const TileTable &tt, const int64_t *rb_off, int64_t n_rb, int32_t n_elem,
                          const int64_t *diag_blk, const int64_t *next_blk, const uint32_t *bitmask,
                          const int32_t *count, int32_t min_pts, int32_t *parent, hipStream_t s);
hipError_t launch_cc_flatten(const int32_t *count, int32_t min_pts, int32_t *parent,
                             uint8_t *isroot, int64_t n_slots, hipStream_t s);
hipError_t launch_fill_i32(int32_t *a, int64_t n, int32_t v, hipStream_t s);
// Roots (isroot, rank = exclusive scan of isroot) keyed for the canonical
// node order: keys[rank] = element << 32 | smallest core point id of the
// component, vals[rank] = rank (minpt: n ints of work space).
hipError_t launch_root_keys(const int32_t *count, int32_t min_pts, const int32_t *parent,
                           const uint32_t *slot_point, const uint8_t *isroot, const int64_t *rank,
                           const uint64_t *slot_elem, int32_t *minpt, uint64_t *keys, uint32_t *vals,
                           int64_t n_slots, hipStream_t s);
// From the N root keys sorted: node_of_rank, node_elem, and node[slot] for
// every slot (NOISE for non-core slots; border slots are set later).
hipError_t launch_node_ids(const int32_t *count, int32_t min_pts, const int32_t *parent, const int64_t *rank,
                           const uint64_t *sorted_keys, const uint32_t *sorted_vals, int64_t N,
                           int32_t *node_of_rank, int32_t *node, int32_t *node_elem, int64_t n_slots,
                           hipStream_t s);
hipError_t launch_noncore_flags(const int32_t *count, int32_t min_pts, const uint64_t *slot_elem,
                                const int64_t *elem_off, const int64_t *rb_off, uint8_t *flag,
                                int64_t n, hipStream_t s);
hipError_t launch_border(const TileTable &tt, const uint32_t *bitmask, const int32_t *count,
                         int32_t min_pts, const uint8_t *ncflag, const int64_t *rb_off,
                         int32_t *node, hipStream_t s);
// keys = node << pbits | point, vals = point (point ids < 2^pbits)
hipError_t launch_member_pairs(const int32_t *node, const uint32_t *slot_point,
                               const int64_t *pos, int64_t n_slots, int pbits, uint64_t *keys,
                               uint32_t *vals, hipStream_t s);
hipError_t launch_flag_labelled(const int32_t *node, uint8_t *flag, int64_t n_slots, hipStream_t s);
hipError_t launch_edge_counts(const uint64_t *pt_keys, int64_t m, int32_t *pairs_per_item,
                              hipStream_t s);
hipError_t launch_edge_emit(const uint64_t *pt_keys, const uint32_t *pt_nodes, int64_t m,
                            const int64_t *pos, int64_t n_nodes, uint64_t *ekeys, hipStream_t s);
hipError_t launch_run_starts(const uint64_t *keys, int64_t m, uint8_t *flag, hipStream_t s);
hipError_t launch_edge_compact(const uint64_t *keys, int64_t m, const int64_t *rank,
                               int64_t n_nodes, int32_t *edges, int32_t *weights, hipStream_t s);
hipError_t launch_node_offsets_from_sorted(const uint64_t *keys, int64_t m, int64_t n_nodes,
                                           int64_t *node_off, hipStream_t s);
hipError_t launch_widen_u32(const uint32_t *in, uint64_t *out, int64_t n, hipStream_t s);
hipError_t launch_narrow_u64(const uint64_t *in, uint32_t *out, int64_t n, hipStream_t s);
hipError_t launch_u32_to_i32(const uint32_t *in, int32_t *out, int64_t n, hipStream_t s);

}  // namespace mgpu
