// graph.hip -- DBSCAN clusters from the adjacency bitmask, and the mapper graph.
//
// Clusters (DBSCAN, Ester et al.): connected components of the core points
// under the eps-neighbour relation, computed with a lock-free union-find whose
// roots are the smallest slot of each component (hooking always attaches the
// larger root under the smaller).  One wave checks one bitmask block (128 x
// 128 bits) against the current labels with ballots and only queues merges
// for rows that join different labels; the queued merges are applied by all
// lanes at once (see k_cc_tiles).
//
// Border points: a non-core point with core neighbours joins the lowest node
// id among them (atomicMin over the same blocks).  Nodes are numbered by
// (element, smallest core point id): the roots, listed by a scan over root
// flags, are sorted by that key.
//
// Edges (nerve of the clusters): (node, point) pairs are sorted by point with
// a stable radix sort, each point emits the node pairs it joins, and a sort
// plus run-length pass gives the edges in lexicographic order with weights.
#include "internal.h"

namespace mgpu {

namespace {

constexpr int32_t NOISE = 0x7fffffff;

__device__ __forceinline__ int32_t ld_rel(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x with path halving.  Parents only ever move to smaller indices of
// the same set, so a stale read is still an ancestor and the loop ends.
__device__ __forceinline__ int32_t uf_find(int32_t *P, int32_t x) {
    while (true) {
        const int32_t p = ld_rel(&P[x]);
        if (p == x) return x;
        const int32_t gp = ld_rel(&P[p]);
        if (gp == p) return p;
        __hip_atomic_store(&P[x], gp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        x = gp;
    }
}

// Merge the sets of a and b; returns a representative of the merged set.
__device__ int32_t uf_union(int32_t *P, int32_t a, int32_t b) {
    while (true) {
        a = uf_find(P, a);
        b = uf_find(P, b);
        if (a == b) return a;
        if (a > b) { const int32_t t = a; a = b; b = t; }
        const int32_t old = atomicCAS(&P[b], b, a);
        if (old == b) return a;
        b = old;
    }
}

struct WaveTile {
    int64_t ne, slot0, blk;
    int e, I, J;
    bool ok;
};

__device__ __forceinline__ WaveTile wave_decode(const TileTable &t, int64_t item) {
    WaveTile r;
    r.ok = item < t.n_items;
    if (!r.ok) return r;
    const TilePos p = tile_lookup(t, item);
    r.ne = p.ne;
    r.slot0 = p.slot0;
    r.blk = p.blk;
    r.e = p.e;
    r.I = p.I;
    r.J = p.J;
    return r;
}

// Logical 4-wave blocks for n items (a multiple of 8); the item of wave w of
// the block, XCD-aware like the tile launch (n: no item).
__host__ __device__ inline int64_t wave_block_count(int64_t n) { return 8 * (((n + 3) / 4 + 7) / 8); }

__device__ __forceinline__ int64_t wave_item(int64_t n, int w) {
    const int64_t G = wave_block_count(n);
    const int64_t bl = block_linear();
    if (bl >= G) return n;
    const int64_t per = G / 8;
    return ((bl % 8) * per + bl / 8) * 4 + w;
}

// One wave per bitmask block; lane l holds the block's rows 2l and 2l+1 (8
// words), their labels, and the labels of columns l and l+64.  Labels come
// from the global union-find at the start (any ancestor will do).
//
// A block is consistent when every core-core bit joins two equal labels.  For
// each distinct column label L the wave builds the 128-bit mask of columns
// labelled L with two ballots; each lane then checks its two rows against the
// mask of its own row label, all lanes at once.  Only rows that fail go
// through the merge step: the row's label and every differing neighbour label
// are merged into the smallest one in registers, and the merges are queued in
// LDS and applied to the global union-find by all lanes in parallel.  Rounds
// repeat until the block is consistent (each failing round merges labels).
constexpr int CC_QCAP = 256;

// The 64-bit value v held by lane `src` (readlane returns a signed 32-bit
// int, so each half is widened as unsigned).
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ void cc_flush(int32_t *parent, int2 *q, int &nq) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    for (int i = (threadIdx.x & (WAVE - 1)); i < nq; i += WAVE) uf_union(parent, q[i].x, q[i].y);
    nq = 0;
}

__device__ void cc_block(const WaveTile &tl, const uint32_t *bitmask, const int32_t *count,
                         int32_t min_pts, int32_t *parent, int2 *Q) {
    const int lane = threadIdx.x & (WAVE - 1);
    int nq = 0;
    constexpr int32_t BIG = 0x7fffffff;
    const int64_t rowbase = tl.slot0 + (int64_t)tl.I * TILE;
    const int64_t colbase = tl.slot0 + (int64_t)tl.J * TILE;
    // labels: lab[0], lab[1] = rows 2l, 2l+1; lab[2], lab[3] = columns l, l+64
    int32_t lab[4];
    bool cr[2];
    uint64_t cc[2];
    // the block's first loads at once: counts, parents (the first hop of
    // each label chain; the parents were compressed before this kernel) and
    // the bitmask block
    int32_t cnt[4], par[4];
    bool valid[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int64_t loc = q < 2 ? (int64_t)tl.I * TILE + 2 * lane + q : (int64_t)tl.J * TILE + lane + 64 * (q - 2);
        valid[q] = loc < tl.ne;
        const int64_t sl = tl.slot0 + (valid[q] ? loc : 0);
        cnt[q] = count[sl];
        par[q] = parent[sl];
    }
    uint32_t wd[8];
    {
        const uint4 *src = (const uint4 *)(bitmask + (uint64_t)tl.blk * TILE_WORDS) + 2 * lane;
        const uint4 u0 = src[0], u1 = src[1];
        wd[0] = u0.x; wd[1] = u0.y; wd[2] = u0.z; wd[3] = u0.w;
        wd[4] = u1.x; wd[5] = u1.y; wd[6] = u1.z; wd[7] = u1.w;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool c = valid[q] && cnt[q] >= min_pts;
        // the label: the current root (any ancestor would be correct, but a
        // stale one makes the block look inconsistent and costs merge rounds)
        int32_t x = par[q];
        if (c) {
            int32_t p2 = parent[x];
            while (p2 != x) {
                x = p2;
                p2 = parent[x];
            }
        }
        lab[q] = c ? x : -1;
        if (q < 2) cr[q] = c; else cc[q - 2] = __ballot(c);
    }
    if (__ballot(cr[0] || cr[1]) == 0 || (cc[0] | cc[1]) == 0) return;
    // core-core bits of my two rows (columns 0..63 and 64..127)
    const uint64_t b00 = cr[0] ? ((((uint64_t)wd[1] << 32) | wd[0]) & cc[0]) : 0;
    const uint64_t b01 = cr[0] ? ((((uint64_t)wd[3] << 32) | wd[2]) & cc[1]) : 0;
    const uint64_t b10 = cr[1] ? ((((uint64_t)wd[5] << 32) | wd[4]) & cc[0]) : 0;
    const uint64_t b11 = cr[1] ? ((((uint64_t)wd[7] << 32) | wd[6]) & cc[1]) : 0;
    for (;;) {
        // masks of the columns that carry each of my row labels
        uint64_t m00 = 0, m01 = 0, m10 = 0, m11 = 0;
        uint64_t p0 = cc[0], p1 = cc[1];
        while (p0 | p1) {
            const int32_t L = p0 ? __builtin_amdgcn_readlane(lab[2], __ffsll((long long)p0) - 1)
                                 : __builtin_amdgcn_readlane(lab[3], __ffsll((long long)p1) - 1);
            const uint64_t e0 = __ballot(lab[2] == L) & cc[0], e1 = __ballot(lab[3] == L) & cc[1];
            if (lab[0] == L) { m00 = e0; m01 = e1; }
            if (lab[1] == L) { m10 = e0; m11 = e1; }
            p0 &= ~e0;
            p1 &= ~e1;
        }
        const uint64_t v0 = __ballot(((b00 & ~m00) | (b01 & ~m01)) != 0);   // row 2l fails
        const uint64_t v1 = __ballot(((b10 & ~m10) | (b11 & ~m11)) != 0);   // row 2l+1 fails
        if ((v0 | v1) == 0) break;
        // merge step for every failing row
        uint64_t todo0 = v0, todo1 = v1;
        while (todo0 | todo1) {
            int src, half;
            if (todo0) { src = __ffsll((long long)todo0) - 1; half = 0; todo0 &= todo0 - 1; }
            else { src = __ffsll((long long)todo1) - 1; half = 1; todo1 &= todo1 - 1; }
            const int r = 2 * src + half;
            const uint64_t r0 = half ? lane_u64(b10, src) : lane_u64(b00, src);
            const uint64_t r1 = half ? lane_u64(b11, src) : lane_u64(b01, src);
            const int32_t lr = __builtin_amdgcn_readlane(half ? lab[1] : lab[0], src);
            int32_t c0 = (((r0 >> lane) & 1ull) && lab[2] != lr) ? lab[2] : BIG;
            int32_t c1 = (((r1 >> lane) & 1ull) && lab[3] != lr) ? lab[3] : BIG;
            if (__ballot(c0 != BIG || c1 != BIG) == 0) continue;
            int32_t mn = min(c0, c1);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mn = min(mn, __shfl_xor(mn, o, WAVE));
            mn = min(mn, lr);
            while (true) {
                const int32_t cand = c0 != BIG ? c0 : c1;
                const uint64_t act = __ballot(cand != BIG);
                if (act == 0) break;
                const int32_t o = __builtin_amdgcn_readlane(cand, __ffsll((long long)act) - 1);
                if (o != mn) {
                    if (lane == 0) Q[nq] = make_int2(mn, o);
                    ++nq;
#pragma unroll
                    for (int q = 0; q < 4; ++q) lab[q] = lab[q] == o ? mn : lab[q];
                }
                c0 = c0 == o ? BIG : c0;
                c1 = c1 == o ? BIG : c1;
            }
            if (lr != mn) {
                if (lane == 0) Q[nq] = make_int2(mn, lr);
                ++nq;
#pragma unroll
                for (int q = 0; q < 4; ++q) lab[q] = lab[q] == lr ? mn : lab[q];
            }
            if (nq > CC_QCAP - 130) cc_flush(parent, Q, nq);
            (void)r;
        }
    }
    cc_flush(parent, Q, nq);
    (void)rowbase;
    (void)colbase;
}

__global__ void __launch_bounds__(256) k_cc_tiles(TileTable tt, const uint32_t *bitmask,
                                                  const int32_t *count, int32_t min_pts,
                                                  int32_t *parent) {
    __shared__ int2 queue[4][CC_QCAP];
    const int w = threadIdx.x / WAVE;
    const WaveTile tl = wave_decode(tt, wave_item(tt.n_items, w));
    if (!tl.ok) return;
    cc_block(tl, bitmask, count, min_pts, parent, queue[w]);
}

// Hooking pass before k_cc_tiles (the sampling idea of Afforest, Sutton et
// al.): for every row block I of every element, the diagonal block (I, I) is
// merged completely, and each core point of row block I + 1 is hung under
// its first core neighbour in row block I (block (I, I + 1)).  Consecutive
// row blocks of one cluster are chained, so dense clusters reach k_cc_tiles
// as single trees and nearly every block there passes its label check
// without merges, in point order and in the cells' locality order alike.
// One wave per row block; `rb_off` numbers the row blocks of all elements.
// diag_blk / next_blk: the blocks of (I, I) and (I, I + 1) at rb_off[e] + I
// (-1: not computed), or null to locate them in the full table.
__global__ void __launch_bounds__(256) k_cc_hook(TileTable tt, const int64_t *rb_off, int64_t n_rb,
                                                 int32_t n_elem, const int64_t *diag_blk, const int64_t *next_blk,
                                                 const uint32_t *bitmask, const int32_t *count, int32_t min_pts,
                                                 int32_t *parent) {
    __shared__ int2 queue[4][CC_QCAP];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const int64_t k = (int64_t)blockIdx.x * 4 + w;
    if (k >= n_rb) return;
    int lo = 0, hi = n_elem;                          // element with rb_off[e] <= k < rb_off[e+1]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (rb_off[mid] <= k) lo = mid; else hi = mid;
    }
    const int e = lo;
    WaveTile tl;
    tl.ok = true;
    tl.e = e;
    tl.I = (int)(k - rb_off[e]);
    tl.J = tl.I;
    tl.slot0 = tt.elem_off[e];
    tl.ne = tt.elem_off[e + 1] - tl.slot0;
    const int64_t T = (tl.ne + TILE - 1) / TILE;
    if (tl.ne <= 0 || tl.I >= T) return;
    const int64_t *cp = tt.colpre + tt.cp_off[e];
    // (I, I): merged completely
    tl.blk = diag_blk ? diag_blk[k] : tt.blk_off[e] + tile_local_index(cp, T, tt.super, tl.I, tl.I);
    if (tl.blk >= 0) cc_block(tl, bitmask, count, min_pts, parent, queue[w]);
    if (tl.I + 1 >= T) return;
    // (I, I + 1): each core column point hung under its first core row neighbour
    tl.J = tl.I + 1;
    tl.blk = next_blk ? next_blk[k] : tt.blk_off[e] + tile_local_index(cp, T, tt.super, tl.I, tl.J);
    if (tl.blk < 0) return;                           // screened out: no neighbours to hook
    // lane holds rows 2l, 2l+1 (words) and columns l, l+64
    uint32_t wd[8];
    {
        const uint4 *src = (const uint4 *)(bitmask + (uint64_t)tl.blk * TILE_WORDS) + 2 * lane;
        const uint4 u0 = src[0], u1 = src[1];
        wd[0] = u0.x; wd[1] = u0.y; wd[2] = u0.z; wd[3] = u0.w;
        wd[4] = u1.x; wd[5] = u1.y; wd[6] = u1.z; wd[7] = u1.w;
    }
    const int64_t rowbase = (int64_t)tl.I * TILE, colloc = (int64_t)tl.J * TILE;
    bool rc[2], ccore[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int64_t r = rowbase + 2 * lane + q;
        rc[q] = r < tl.ne && count[tl.slot0 + r] >= min_pts;
        const int64_t c = colloc + lane + 64 * q;
        ccore[q] = c < tl.ne && count[tl.slot0 + c] >= min_pts;
    }
    const uint64_t rc0 = __ballot(rc[0]), rc1 = __ballot(rc[1]);   // rows 2l and 2l+1
    int32_t first0 = -1, first1 = -1;                             // first core row per column
    for (int r = 0; r < TILE; ++r) {
        const int src = r >> 1;
        if (!((((r & 1) ? rc1 : rc0) >> src) & 1ull)) continue;
        uint32_t x0, x1, x2, x3;
        if (r & 1) {
            x0 = __builtin_amdgcn_readlane(wd[4], src); x1 = __builtin_amdgcn_readlane(wd[5], src);
            x2 = __builtin_amdgcn_readlane(wd[6], src); x3 = __builtin_amdgcn_readlane(wd[7], src);
        } else {
            x0 = __builtin_amdgcn_readlane(wd[0], src); x1 = __builtin_amdgcn_readlane(wd[1], src);
            x2 = __builtin_amdgcn_readlane(wd[2], src); x3 = __builtin_amdgcn_readlane(wd[3], src);
        }
        const uint32_t lw = lane < 32 ? x0 : x1, hw = lane < 32 ? x2 : x3;
        if (first0 < 0 && ((lw >> (lane & 31)) & 1u)) first0 = r;
        if (first1 < 0 && ((hw >> (lane & 31)) & 1u)) first1 = r;
        if (__ballot((ccore[0] && first0 < 0) || (ccore[1] && first1 < 0)) == 0) break;
    }
    const int64_t rowslot = tl.slot0 + rowbase, colslot = tl.slot0 + colloc;
    if (ccore[0] && first0 >= 0) uf_union(parent, (int32_t)(rowslot + first0), (int32_t)(colslot + lane));
    if (ccore[1] && first1 >= 0) uf_union(parent, (int32_t)(rowslot + first1), (int32_t)(colslot + lane + 64));
}

__global__ void k_cc_init(int32_t *parent, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) parent[i] = (int32_t)i;
}

// parent[i] = the root of i (path compression before the block pass).
__global__ void k_cc_compress(int32_t *parent, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int32_t r = uf_find(parent, (int32_t)i);
        if (r != (int32_t)i) __hip_atomic_store(&parent[i], r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Root of x without writes.  After the last union the forest is fixed, and
// k_cc_flatten must leave every core parent at its root: a path-halving store
// of another thread (uf_find), computed from a pointer it read before this
// thread's store, could otherwise land after it and put a non-root ancestor
// back, and k_node_ids would then give the point the cluster id of another
// root.
__device__ __forceinline__ int32_t uf_root(const int32_t *P, int32_t x) {
    int32_t p = ld_rel(&P[x]);
    while (p != x) {
        x = p;
        p = ld_rel(&P[x]);
    }
    return x;
}

__global__ void k_cc_flatten(const int32_t *count, int32_t min_pts, int32_t *parent,
                             uint8_t *isroot, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (count[i] >= min_pts) {
        const int32_t r = uf_root(parent, (int32_t)i);
        parent[i] = r;
        isroot[i] = r == (int32_t)i;
    } else {
        isroot[i] = 0;
    }
}

// Canonical cluster numbering.  Slots are laid out by (element, cell), not
// by point id, so the root of a component (its smallest slot) need not hold
// its smallest core point: nodes are numbered by sorting the roots by
// (element, smallest core point id), as the labelling rule asks.
__global__ void k_fill_i32(int32_t *a, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) a[i] = v;
}

// minpt[r] = the smallest point id among the core slots whose root is r.
// A core slot whose predecessor is a core slot of the same component with a
// smaller point id cannot hold the minimum (points ascend within a cell's
// run of slots), so only the other slots take part: far fewer atomics on
// the same root.
__global__ void k_root_minpt(const int32_t *count, int32_t min_pts, const int32_t *parent,
                             const uint32_t *slot_point, int32_t *minpt, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || count[i] < min_pts) return;
    const int32_t r = parent[i];
    if (i > 0 && count[i - 1] >= min_pts && parent[i - 1] == r && slot_point[i - 1] < slot_point[i]) return;
    atomicMin(&minpt[r], (int32_t)slot_point[i]);
}

// Root of rank r (roots counted in slot order): key (element, minpt), value r.
__global__ void k_root_keys(const uint8_t *isroot, const int64_t *rank, const uint64_t *slot_elem,
                            const int32_t *minpt, uint64_t *keys, uint32_t *vals, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || !isroot[i]) return;
    const int64_t r = rank[i];
    keys[r] = (slot_elem[i] << 32) | (uint64_t)(uint32_t)minpt[i];
    vals[r] = (uint32_t)r;
}

// After the sort by key: the node id of root rank vals[p] is p.
__global__ void k_root_order(const uint64_t *keys, const uint32_t *vals, int64_t N, int32_t *node_of_rank,
                             int32_t *node_elem) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= N) return;
    node_of_rank[vals[p]] = (int32_t)p;
    node_elem[p] = (int32_t)(keys[p] >> 32);
}

__global__ void k_node_ids(const int32_t *count, int32_t min_pts, const int32_t *parent,
                           const int64_t *rank, const int32_t *node_of_rank, int32_t *node, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    node[i] = count[i] >= min_pts ? node_of_rank[rank[parent[i]]] : NOISE;
}

// flag[rb] = 1 if the 128-slot row block rb (row blocks numbered per element,
// rb_off[e] + local / 128) holds a non-core member
__global__ void k_noncore_flags(const int32_t *count, int32_t min_pts, const uint64_t *slot_elem,
                                const int64_t *elem_off, const int64_t *rb_off, uint8_t *flag,
                                int64_t n) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= n || count[s] >= min_pts) return;
    const int64_t e = (int64_t)slot_elem[s];
    flag[rb_off[e] + (s - elem_off[e]) / TILE] = 1;
}

__global__ void __launch_bounds__(256) k_border(TileTable tt, const uint32_t *bitmask,
                                                const int32_t *count, int32_t min_pts,
                                                const uint8_t *ncflag, const int64_t *rb_off,
                                                int32_t *node) {
    __shared__ uint32_t words[4][TILE_WORDS];
    __shared__ int32_t nid[4][2 * TILE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const WaveTile tl = wave_decode(tt, wave_item(tt.n_items, w));
    if (!tl.ok) return;
    if (!ncflag[rb_off[tl.e] + tl.I] && !ncflag[rb_off[tl.e] + tl.J]) return;   // all core
    uint64_t coreI[2], coreJ[2], ncI[2], ncJ[2];
    int32_t *N = nid[w];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = lane + 64 * q;
        const int64_t loc = (t < TILE ? (int64_t)tl.I * TILE + t : (int64_t)tl.J * TILE + (t - TILE));
        const bool valid = loc < tl.ne;
        const bool core = valid && count[tl.slot0 + loc] >= min_pts;
        N[t] = core ? node[tl.slot0 + loc] : NOISE;
        const uint64_t mc = __ballot(core), mn = __ballot(valid && !core);
        if (q < 2) { coreI[q] = mc; ncI[q] = mn; } else { coreJ[q - 2] = mc; ncJ[q - 2] = mn; }
    }
    // only blocks with a core point on one side and a non-core point on the other matter
    const bool rows_nc = (ncI[0] | ncI[1]) && (coreJ[0] | coreJ[1]);
    const bool cols_nc = (ncJ[0] | ncJ[1]) && (coreI[0] | coreI[1]);
    if (!rows_nc && !cols_nc) return;
    uint32_t *W = words[w];
    {
        const uint4 *src = (const uint4 *)(bitmask + (uint64_t)tl.blk * TILE_WORDS);
        ((uint4 *)W)[lane] = src[lane];
        ((uint4 *)W)[lane + 64] = src[lane + 64];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    // non-core rows r: the lowest node among their core neighbour columns.
    // Few of them: one pass per row (lane l checks columns l and l + 64);
    // many: lane l takes rows l and l + 64 and walks the core columns among
    // its row's own neighbours.
    const int64_t rowbase = tl.slot0 + (int64_t)tl.I * TILE;
    if (rows_nc && __popcll(ncI[0]) + __popcll(ncI[1]) > 16) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if ((ncI[h] >> lane) & 1ull) {
                const int r = 64 * h + lane;
                const uint4 rw = ((const uint4 *)W)[r];   // the row's four words
                uint64_t m0 = ((((uint64_t)rw.y) << 32) | rw.x) & coreJ[0];
                uint64_t m1 = ((((uint64_t)rw.w) << 32) | rw.z) & coreJ[1];
                int32_t m = NOISE;
                while (m0) {
                    m = min(m, N[TILE + __ffsll((long long)m0) - 1]);
                    m0 &= m0 - 1;
                }
                while (m1) {
                    m = min(m, N[TILE + 64 + __ffsll((long long)m1) - 1]);
                    m1 &= m1 - 1;
                }
                if (m != NOISE) atomicMin(&node[rowbase + r], m);
            }
        }
    } else if (rows_nc) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint64_t todo = ncI[h];
            while (todo) {
                const int r = 64 * h + __ffsll((long long)todo) - 1;
                todo &= todo - 1;
                const uint32_t wa = W[r * 4 + (lane >> 5)], wb = W[r * 4 + 2 + (lane >> 5)];
                int32_t m = NOISE;
                if (((wa >> (lane & 31)) & 1u) && ((coreJ[0] >> lane) & 1ull)) m = N[TILE + lane];
                if (((wb >> (lane & 31)) & 1u) && ((coreJ[1] >> lane) & 1ull)) m = min(m, N[TILE + 64 + lane]);
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, WAVE));
                if (lane == 0 && m != NOISE) atomicMin(&node[rowbase + r], m);
            }
        }
    }
    // non-core columns c: the lowest node among their core neighbour rows.
    // Few of them: one pass per column (lane l checks rows l and l + 64);
    // many: one scan over the core rows, each lane keeping its two columns'
    // minima.
    const int64_t colbase = tl.slot0 + (int64_t)tl.J * TILE;
    if (cols_nc && __popcll(ncJ[0]) + __popcll(ncJ[1]) <= 16) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint64_t todo = ncJ[h];
            while (todo) {
                const int c = 64 * h + __ffsll((long long)todo) - 1;
                todo &= todo - 1;
                const int wc = c >> 5;
                const uint32_t bit = 1u << (c & 31);
                int32_t m = NOISE;
                if ((W[lane * 4 + wc] & bit) && ((coreI[0] >> lane) & 1ull)) m = N[lane];
                if ((W[(lane + 64) * 4 + wc] & bit) && ((coreI[1] >> lane) & 1ull)) m = min(m, N[64 + lane]);
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, WAVE));
                if (lane == 0 && m != NOISE) atomicMin(&node[colbase + c], m);
            }
        }
    } else if (cols_nc) {
        int32_t cmin0 = NOISE, cmin1 = NOISE;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            uint64_t todo = coreI[h];
            while (todo) {
                const int r = 64 * h + __ffsll((long long)todo) - 1;
                todo &= todo - 1;
                const uint32_t wa = W[r * 4 + (lane >> 5)], wb = W[r * 4 + 2 + (lane >> 5)];
                const int32_t rn = N[r];
                if (((wa >> (lane & 31)) & 1u) && ((ncJ[0] >> lane) & 1ull)) cmin0 = min(cmin0, rn);
                if (((wb >> (lane & 31)) & 1u) && ((ncJ[1] >> lane) & 1ull)) cmin1 = min(cmin1, rn);
            }
        }
        if (cmin0 != NOISE) atomicMin(&node[colbase + lane], cmin0);
        if (cmin1 != NOISE) atomicMin(&node[colbase + 64 + lane], cmin1);
    }
}

__global__ void k_flag_labelled(const int32_t *node, uint8_t *flag, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = node[i] != NOISE;
}

// (node, point) pairs keyed node << pbits | point: sorted, each node's
// members come out in ascending point order whatever the slot order.
__global__ void k_member_pairs(const int32_t *node, const uint32_t *slot_point, const int64_t *pos,
                               int64_t n, int pbits, uint64_t *keys, uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || node[i] == NOISE) return;
    keys[pos[i]] = ((uint64_t)node[i] << pbits) | (uint64_t)slot_point[i];
    vals[pos[i]] = slot_point[i];
}

__global__ void k_edge_counts(const uint64_t *pk, int64_t m, int32_t *cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (i > 0 && pk[i - 1] == pk[i]) { cnt[i] = 0; return; }
    int64_t e = i + 1;
    while (e < m && pk[e] == pk[i]) ++e;
    const int64_t c = e - i;
    cnt[i] = (int32_t)(c * (c - 1) / 2);
}

__global__ void k_edge_emit(const uint64_t *pk, const uint32_t *pn, int64_t m, const int64_t *pos,
                            int64_t nn, uint64_t *ek) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    if (i > 0 && pk[i - 1] == pk[i]) return;
    int64_t e = i + 1;
    while (e < m && pk[e] == pk[i]) ++e;
    int64_t o = pos[i];
    for (int64_t x = i; x < e; ++x)
        for (int64_t y = x + 1; y < e; ++y) ek[o++] = (uint64_t)pn[x] * (uint64_t)nn + (uint64_t)pn[y];
}

__global__ void k_run_starts(const uint64_t *k, int64_t m, uint8_t *flag) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) flag[i] = (i == 0 || k[i - 1] != k[i]);
}

// Run r of the sorted edge keys starts at i (rank[i] = r, the exclusive scan
// of the run-start flags, m + 1 entries) and ends where run r + 1 starts:
// the first j > i with rank[j] = r + 2 is one past that start (or m when r
// is the last run).  A binary search, so a heavy edge costs no long walk.
__global__ void k_edge_compact(const uint64_t *k, int64_t m, const int64_t *rank, int64_t nn,
                               int32_t *edges, int32_t *weights) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m || (i > 0 && k[i - 1] == k[i])) return;
    const int64_t r = rank[i];
    int64_t lo = i + 1, hi = m + 1;             // first j in [i + 1, m] with rank[j] >= r + 2, else m + 1
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (rank[mid] >= r + 2) hi = mid; else lo = mid + 1;
    }
    const int64_t e = lo - 1;
    edges[2 * r] = (int32_t)(k[i] / (uint64_t)nn);
    edges[2 * r + 1] = (int32_t)(k[i] % (uint64_t)nn);
    weights[r] = (int32_t)(e - i);
}

__global__ void k_node_offsets(const uint64_t *k, int64_t m, int64_t nn, int64_t *off) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v > nn) return;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (k[mid] < (uint64_t)v) lo = mid + 1; else hi = mid;
    }
    off[v] = lo;
}

__global__ void k_widen_u32(const uint32_t *in, uint64_t *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = in[i];
}

__global__ void k_narrow_u64(const uint64_t *in, uint32_t *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (uint32_t)in[i];
}

__global__ void k_u32_to_i32(const uint32_t *in, int32_t *out, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (int32_t)in[i];
}

inline unsigned nblk(int64_t n, int b = 256) { return (unsigned)((n + b - 1) / b); }

inline dim3 wave_blocks(int64_t items) { return grid_2d(wave_block_count(items)); }

}  // namespace

hipError_t launch_cc_compress(int32_t *parent, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_cc_compress<<<dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s>>>(parent, n);
    return hipGetLastError();
}

hipError_t launch_cc_init(int32_t *parent, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_cc_init<<<nblk(n), 256, 0, s>>>(parent, n);
    return hipGetLastError();
}

hipError_t launch_cc_tiles(const TileTable &tt, const uint32_t *bitmask, const int32_t *count,
                           int32_t min_pts, int32_t *parent, hipStream_t s) {
    if (tt.n_items <= 0) return hipSuccess;
    k_cc_tiles<<<wave_blocks(tt.n_items), 256, 0, s>>>(tt, bitmask, count, min_pts, parent);
    return hipGetLastError();
}

hipError_t launch_cc_hook(const TileTable &tt, const int64_t *rb_off, int64_t n_rb, int32_t n_elem,
                          const int64_t *diag_blk, const int64_t *next_blk, const uint32_t *bitmask,
                          const int32_t *count, int32_t min_pts, int32_t *parent, hipStream_t s) {
    if (n_rb <= 0) return hipSuccess;
    k_cc_hook<<<dim3((unsigned)((n_rb + 3) / 4)), 256, 0, s>>>(tt, rb_off, n_rb, n_elem, diag_blk, next_blk,
                                                               bitmask, count, min_pts, parent);
    return hipGetLastError();
}

hipError_t launch_cc_flatten(const int32_t *count, int32_t min_pts, int32_t *parent,
                             uint8_t *isroot, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_cc_flatten<<<nblk(n), 256, 0, s>>>(count, min_pts, parent, isroot, n);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t *a, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<nblk(n), 256, 0, s>>>(a, n, v);
    return hipGetLastError();
}

hipError_t launch_root_keys(const int32_t *count, int32_t min_pts, const int32_t *parent,
                           const uint32_t *slot_point, const uint8_t *isroot, const int64_t *rank,
                           const uint64_t *slot_elem, int32_t *minpt, uint64_t *keys, uint32_t *vals,
                           int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_i32<<<nblk(n), 256, 0, s>>>(minpt, n, 0x7fffffff);
    k_root_minpt<<<nblk(n), 256, 0, s>>>(count, min_pts, parent, slot_point, minpt, n);
    k_root_keys<<<nblk(n), 256, 0, s>>>(isroot, rank, slot_elem, minpt, keys, vals, n);
    return hipGetLastError();
}

hipError_t launch_node_ids(const int32_t *count, int32_t min_pts, const int32_t *parent, const int64_t *rank,
                           const uint64_t *sorted_keys, const uint32_t *sorted_vals, int64_t N,
                           int32_t *node_of_rank, int32_t *node, int32_t *node_elem, int64_t n, hipStream_t s) {
    if (N > 0) k_root_order<<<nblk(N), 256, 0, s>>>(sorted_keys, sorted_vals, N, node_of_rank, node_elem);
    if (n > 0) k_node_ids<<<nblk(n), 256, 0, s>>>(count, min_pts, parent, rank, node_of_rank, node, n);
    return hipGetLastError();
}

hipError_t launch_noncore_flags(const int32_t *count, int32_t min_pts, const uint64_t *slot_elem,
                                const int64_t *elem_off, const int64_t *rb_off, uint8_t *flag,
                                int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_noncore_flags<<<nblk(n), 256, 0, s>>>(count, min_pts, slot_elem, elem_off, rb_off, flag, n);
    return hipGetLastError();
}

hipError_t launch_border(const TileTable &tt, const uint32_t *bitmask, const int32_t *count,
                         int32_t min_pts, const uint8_t *ncflag, const int64_t *rb_off,
                         int32_t *node, hipStream_t s) {
    if (tt.n_items <= 0) return hipSuccess;
    k_border<<<wave_blocks(tt.n_items), 256, 0, s>>>(tt, bitmask, count, min_pts, ncflag, rb_off, node);
    return hipGetLastError();
}

hipError_t launch_flag_labelled(const int32_t *node, uint8_t *flag, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_flag_labelled<<<nblk(n), 256, 0, s>>>(node, flag, n);
    return hipGetLastError();
}

hipError_t launch_member_pairs(const int32_t *node, const uint32_t *slot_point, const int64_t *pos,
                               int64_t n, int pbits, uint64_t *keys, uint32_t *vals, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_member_pairs<<<nblk(n), 256, 0, s>>>(node, slot_point, pos, n, pbits, keys, vals);
    return hipGetLastError();
}

hipError_t launch_edge_counts(const uint64_t *pt_keys, int64_t m, int32_t *cnt, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    k_edge_counts<<<nblk(m), 256, 0, s>>>(pt_keys, m, cnt);
    return hipGetLastError();
}

hipError_t launch_edge_emit(const uint64_t *pt_keys, const uint32_t *pt_nodes, int64_t m,
                            const int64_t *pos, int64_t n_nodes, uint64_t *ekeys, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    k_edge_emit<<<nblk(m), 256, 0, s>>>(pt_keys, pt_nodes, m, pos, n_nodes, ekeys);
    return hipGetLastError();
}

hipError_t launch_run_starts(const uint64_t *keys, int64_t m, uint8_t *flag, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    k_run_starts<<<nblk(m), 256, 0, s>>>(keys, m, flag);
    return hipGetLastError();
}

hipError_t launch_edge_compact(const uint64_t *keys, int64_t m, const int64_t *rank,
                               int64_t n_nodes, int32_t *edges, int32_t *weights, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    k_edge_compact<<<nblk(m), 256, 0, s>>>(keys, m, rank, n_nodes, edges, weights);
    return hipGetLastError();
}

hipError_t launch_node_offsets_from_sorted(const uint64_t *keys, int64_t m, int64_t n_nodes,
                                           int64_t *node_off, hipStream_t s) {
    k_node_offsets<<<nblk(n_nodes + 1), 256, 0, s>>>(keys, m, n_nodes, node_off);
    return hipGetLastError();
}

hipError_t launch_widen_u32(const uint32_t *in, uint64_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_widen_u32<<<nblk(n), 256, 0, s>>>(in, out, n);
    return hipGetLastError();
}

hipError_t launch_narrow_u64(const uint64_t *in, uint32_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_narrow_u64<<<nblk(n), 256, 0, s>>>(in, out, n);
    return hipGetLastError();
}

hipError_t launch_u32_to_i32(const uint32_t *in, int32_t *out, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_u32_to_i32<<<nblk(n), 256, 0, s>>>(in, out, n);
    return hipGetLastError();
}

}  // namespace mgpu
