// graph.hip -- DBSCAN clusters from the adjacency bitmask, and the mapper graph.
//
// Clusters (DBSCAN, Ester et al.): connected components of the core points
// under the eps-neighbour relation.  One wave takes one bitmask block (128 x
// 128 bits): it caches the block and a label per row and column in LDS, and
// for every core row tests 64 columns per step with the lanes as bit
// positions.  Only pairs whose cached labels differ reach the global
// union-find (lock-free, hooking the larger root under the smaller, so every
// root ends as its component's smallest slot); after each union the cached
// labels of both merged sets are rewritten, so a dense cluster costs a few
// unions per block instead of one per edge.
//
// Border points: a non-core point with core neighbours joins the lowest node
// id among them (atomicMin over the same blocks).  Nodes are numbered by a
// scan over root flags in slot order, i.e. by (element, smallest core index).
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
    int I, J;
    bool ok;
};

__device__ __forceinline__ WaveTile wave_decode(const TileTable &t, int64_t item) {
    WaveTile r;
    r.ok = item < t.n_items;
    if (!r.ok) return r;
    int lo = 0, hi = t.nord;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (t.item_off[mid] <= item) lo = mid; else hi = mid;
    }
    const int e = t.order[lo];
    const int64_t p = item - t.item_off[lo];
    int64_t J = (int64_t)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
    while ((J + 1) * (J + 2) / 2 <= p) ++J;
    while (J * (J + 1) / 2 > p) --J;
    r.J = (int)J;
    r.I = (int)(p - J * (J + 1) / 2);
    r.slot0 = t.elem_off[e];
    r.ne = t.elem_off[e + 1] - r.slot0;
    r.blk = t.blk_off[e] + p;
    return r;
}

// item for wave w of a 4-wave block, XCD-aware like the tile launch
__device__ __forceinline__ int64_t wave_item(int w) {
    const int64_t G = gridDim.x;
    const int64_t per = (G + 7) / 8;
    const int64_t b = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    return b * 4 + w;
}

__global__ void __launch_bounds__(256) k_cc_tiles(TileTable tt, const uint32_t *bitmask,
                                                  const int32_t *count, int32_t min_pts,
                                                  int32_t *parent) {
    __shared__ uint32_t words[4][TILE_WORDS];
    __shared__ int32_t lab[4][2 * TILE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const WaveTile tl = wave_decode(tt, wave_item(w));
    if (!tl.ok) return;
    uint32_t *W = words[w];
    int32_t *L = lab[w];
    {
        const uint4 *src = (const uint4 *)(bitmask + (uint64_t)tl.blk * TILE_WORDS);
        ((uint4 *)W)[lane] = src[lane];
        ((uint4 *)W)[lane + 64] = src[lane + 64];
    }
    uint64_t coreI[2], coreJ[2];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int t = lane + 64 * q;                   // 0..127 rows, 128..255 columns
        const int64_t loc = (t < TILE ? (int64_t)tl.I * TILE + t : (int64_t)tl.J * TILE + (t - TILE));
        const bool core = loc < tl.ne && count[tl.slot0 + loc] >= min_pts;
        L[t] = core ? uf_find(parent, (int32_t)(tl.slot0 + loc)) : -1;
        const uint64_t m = __ballot(core);
        if (q < 2) coreI[q] = m; else coreJ[q - 2] = m;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (!((coreI[0] | coreI[1]) && (coreJ[0] | coreJ[1]))) return;
    const int64_t colbase = tl.slot0 + (int64_t)tl.J * TILE;
    for (int r = 0; r < TILE; ++r) {
        if (!((coreI[r >> 6] >> (r & 63)) & 1ull)) continue;
        const uint32_t wa = W[r * 4 + (lane >> 5)], wb = W[r * 4 + 2 + (lane >> 5)];
        const bool b0 = ((wa >> (lane & 31)) & 1u) && ((coreJ[0] >> lane) & 1ull);
        const bool b1 = ((wb >> (lane & 31)) & 1u) && ((coreJ[1] >> lane) & 1ull);
        uint64_t m0 = __ballot(b0 && L[r] != L[TILE + lane]);
        uint64_t m1 = __ballot(b1 && L[r] != L[TILE + 64 + lane]);
        while (m0 | m1) {
            const int c = m0 ? __ffsll((long long)m0) - 1 : 64 + __ffsll((long long)m1) - 1;
            const int32_t o1 = L[r], o2 = L[TILE + c];
            int32_t root = 0;
            if (lane == 0) root = uf_union(parent, (int32_t)(tl.slot0 + (int64_t)tl.I * TILE + r),
                                           (int32_t)(colbase + c));
            root = __shfl(root, 0, WAVE);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int t = lane + 64 * q;
                const int32_t v = L[t];
                if (v >= 0 && (v == o1 || v == o2)) L[t] = root;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            m0 = __ballot(b0 && L[r] != L[TILE + lane]);
            m1 = __ballot(b1 && L[r] != L[TILE + 64 + lane]);
        }
    }
}

__global__ void k_cc_init(int32_t *parent, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) parent[i] = (int32_t)i;
}

__global__ void k_cc_flatten(const int32_t *count, int32_t min_pts, int32_t *parent,
                             uint8_t *isroot, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (count[i] >= min_pts) {
        const int32_t r = uf_find(parent, (int32_t)i);
        parent[i] = r;
        isroot[i] = r == (int32_t)i;
    } else {
        isroot[i] = 0;
    }
}

__global__ void k_node_ids(const int32_t *count, int32_t min_pts, const int32_t *parent,
                           const int64_t *rank, const uint64_t *slot_elem, int32_t *node,
                           int32_t *node_elem, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (count[i] >= min_pts) {
        const int32_t r = parent[i];
        node[i] = (int32_t)rank[r];
        if (r == (int32_t)i) node_elem[rank[i]] = (int32_t)slot_elem[i];
    } else {
        node[i] = NOISE;
    }
}

__global__ void __launch_bounds__(256) k_border(TileTable tt, const uint32_t *bitmask,
                                                const int32_t *count, int32_t min_pts,
                                                int32_t *node) {
    __shared__ uint32_t words[4][TILE_WORDS];
    __shared__ int32_t nid[4][2 * TILE];
    const int w = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
    const WaveTile tl = wave_decode(tt, wave_item(w));
    if (!tl.ok) return;
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
    int32_t cmin0 = NOISE, cmin1 = NOISE;
    const int64_t rowbase = tl.slot0 + (int64_t)tl.I * TILE;
    for (int r = 0; r < TILE; ++r) {
        const bool rcore = (coreI[r >> 6] >> (r & 63)) & 1ull;
        const bool rnc = (ncI[r >> 6] >> (r & 63)) & 1ull;
        if (!rcore && !rnc) continue;
        const uint32_t wa = W[r * 4 + (lane >> 5)], wb = W[r * 4 + 2 + (lane >> 5)];
        const bool b0 = (wa >> (lane & 31)) & 1u, b1 = (wb >> (lane & 31)) & 1u;
        if (rnc) {           // non-core row: lowest node among core columns
            int32_t m = NOISE;
            if (b0 && ((coreJ[0] >> lane) & 1ull)) m = N[TILE + lane];
            if (b1 && ((coreJ[1] >> lane) & 1ull)) m = min(m, N[TILE + 64 + lane]);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) m = min(m, __shfl_xor(m, o, WAVE));
            if (lane == 0 && m != NOISE) atomicMin(&node[rowbase + r], m);
        } else {             // core row: non-core columns take its node
            const int32_t rn = N[r];
            if (b0 && ((ncJ[0] >> lane) & 1ull)) cmin0 = min(cmin0, rn);
            if (b1 && ((ncJ[1] >> lane) & 1ull)) cmin1 = min(cmin1, rn);
        }
    }
    const int64_t colbase = tl.slot0 + (int64_t)tl.J * TILE;
    if (cmin0 != NOISE) atomicMin(&node[colbase + lane], cmin0);
    if (cmin1 != NOISE) atomicMin(&node[colbase + 64 + lane], cmin1);
}

__global__ void k_flag_labelled(const int32_t *node, uint8_t *flag, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) flag[i] = node[i] != NOISE;
}

__global__ void k_member_pairs(const int32_t *node, const uint32_t *slot_point, const int64_t *pos,
                               int64_t n, uint64_t *keys, uint32_t *vals) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || node[i] == NOISE) return;
    keys[pos[i]] = (uint64_t)node[i];
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

__global__ void k_edge_compact(const uint64_t *k, int64_t m, const int64_t *rank, int64_t nn,
                               int32_t *edges, int32_t *weights) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m || (i > 0 && k[i - 1] == k[i])) return;
    int64_t e = i + 1;
    while (e < m && k[e] == k[i]) ++e;
    const int64_t r = rank[i];
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

inline unsigned wave_blocks(int64_t items) {
    const int64_t b = (items + 3) / 4;
    return (unsigned)(8 * ((b + 7) / 8));
}

}  // namespace

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

hipError_t launch_cc_flatten(const int32_t *count, int32_t min_pts, int32_t *parent,
                             uint8_t *isroot, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_cc_flatten<<<nblk(n), 256, 0, s>>>(count, min_pts, parent, isroot, n);
    return hipGetLastError();
}

hipError_t launch_node_ids(const int32_t *count, int32_t min_pts, const int32_t *parent,
                           const int64_t *root_rank, const uint64_t *slot_elem, int32_t *node,
                           int32_t *node_elem, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_node_ids<<<nblk(n), 256, 0, s>>>(count, min_pts, parent, root_rank, slot_elem, node, node_elem, n);
    return hipGetLastError();
}

hipError_t launch_border(const TileTable &tt, const uint32_t *bitmask, const int32_t *count,
                         int32_t min_pts, int32_t *node, hipStream_t s) {
    if (tt.n_items <= 0) return hipSuccess;
    k_border<<<wave_blocks(tt.n_items), 256, 0, s>>>(tt, bitmask, count, min_pts, node);
    return hipGetLastError();
}

hipError_t launch_flag_labelled(const int32_t *node, uint8_t *flag, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_flag_labelled<<<nblk(n), 256, 0, s>>>(node, flag, n);
    return hipGetLastError();
}

hipError_t launch_member_pairs(const int32_t *node, const uint32_t *slot_point, const int64_t *pos,
                               int64_t n, uint64_t *keys, uint32_t *vals, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_member_pairs<<<nblk(n), 256, 0, s>>>(node, slot_point, pos, n, keys, vals);
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
