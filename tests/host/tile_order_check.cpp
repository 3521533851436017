// Host check of the tile order that the tile launch, the item table and the
// components kernels share (internal.h): for every supertile size the runtime
// can choose, and for tables of three elements of up to tmax tile rows,
// tile_decode maps the items one to one onto the tile pairs I <= J < T of
// each element, item p of an element owns bitmask block blk_off[e] + p, and
// tile_local_index inverts the decode.  A wrong order would make the kernels
// write another element's bitmask blocks, so this runs on the host only.
//
// usage: tile_order_check [tmax]   prints "ok <items>" and exits 0, or names
// the first failure and exits 1.
#include "internal.h"

#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <set>

using namespace mgpu;

static int check(int64_t S, const std::vector<int64_t> &Trows, int64_t &items) {
    const int64_t E = (int64_t)Trows.size();
    // the runtime's table: elements largest first, bitmask blocks in element order
    std::vector<int32_t> order;
    std::vector<int64_t> P(E), blk_off(E), elem_off(E + 1, 0);
    int64_t nblocks = 0;
    for (int64_t e = 0; e < E; ++e) {
        const int64_t ne = Trows[e] == 0 ? 0 : Trows[e] * TILE - (e % 3) * 37;   // ragged last tile
        elem_off[e + 1] = elem_off[e] + ne;
        P[e] = Trows[e] * (Trows[e] + 1) / 2;
        blk_off[e] = nblocks;
        nblocks += P[e];
        if (ne > 0) order.push_back((int32_t)e);
    }
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return P[a] > P[b]; });
    std::vector<int64_t> item_off(order.size() + 1, 0);
    for (size_t k = 0; k < order.size(); ++k) item_off[k + 1] = item_off[k] + P[order[k]];
    std::vector<int64_t> colpre, cp_off(E);
    build_supertile_columns(Trows, S, colpre, cp_off);
    TileTable tt{};
    tt.item_off = item_off.data();
    tt.order = order.data();
    tt.elem_off = elem_off.data();
    tt.blk_off = blk_off.data();
    tt.colpre = colpre.data();
    tt.cp_off = cp_off.data();
    tt.nord = (int32_t)order.size();
    tt.super = (int32_t)S;
    tt.n_items = nblocks;
    std::vector<char> seen((size_t)nblocks, 0);
    for (int64_t it = 0; it < nblocks; ++it) {
        const TilePos r = tile_decode(tt, it);
        const int64_t T = Trows[r.e];
        const bool ok = r.e >= 0 && r.e < E && r.I >= 0 && r.I <= r.J && r.J < T && r.blk >= 0 &&
                        r.blk < nblocks && !seen[r.blk] && r.slot0 == elem_off[r.e] &&
                        r.ne == elem_off[r.e + 1] - elem_off[r.e] &&
                        blk_off[r.e] + tile_local_index(colpre.data() + cp_off[r.e], T, S, r.I, r.J) == r.blk;
        if (!ok) {
            std::printf("FAIL S=%ld item=%ld e=%d I=%d J=%d blk=%ld\n", (long)S, (long)it, r.e, r.I, r.J,
                        (long)r.blk);
            return 1;
        }
        seen[r.blk] = 1;
        ++items;
    }
    // macro tiles (pairs of 256-row blocks) over the same elements: every tile
    // pair's block is covered by exactly one macro item, at its own (I, J)
    for (int64_t Sm : {1, 2, 4, 8}) {
        std::vector<int64_t> T2(E), mitem_off(order.size() + 1, 0), mcolpre, mcp_off(E);
        for (int64_t e = 0; e < E; ++e) T2[e] = (elem_off[e + 1] - elem_off[e] + MTILE - 1) / MTILE;
        for (size_t k = 0; k < order.size(); ++k) mitem_off[k + 1] = mitem_off[k] + T2[order[k]] * (T2[order[k]] + 1) / 2;
        build_supertile_columns(T2, Sm, mcolpre, mcp_off);
        TileTable mt = tt;
        mt.item_off = mitem_off.data();
        mt.colpre = mcolpre.data();
        mt.cp_off = mcp_off.data();
        mt.super = (int32_t)Sm;
        mt.n_items = mitem_off.back();
        std::vector<char> mseen((size_t)nblocks, 0);
        int64_t covered = 0;
        for (int64_t it = 0; it < mt.n_items; ++it) {
            const MacroItem m = macro_decode(mt, tt, it);
            const int64_t T = Trows[m.e];
            bool ok = m.e >= 0 && m.e < E && m.P <= m.Q && (int64_t)m.Q < T2[m.e] && m.slot0 == elem_off[m.e] &&
                      m.ne == elem_off[m.e + 1] - elem_off[m.e];
            for (int a = 0; a < 2 && ok; ++a)
                for (int b = 0; b < 2 && ok; ++b) {
                    const int64_t I = 2 * m.P + a, J = 2 * m.Q + b, blk = m.blk[2 * a + b];
                    const bool present = I < T && J < T && I <= J;
                    if (!present) { ok = blk == -1; continue; }
                    ok = blk >= 0 && blk < nblocks && !mseen[blk];
                    if (!ok) break;
                    const TilePos r = tile_decode(tt, blk - blk_off[m.e] + item_off[std::find(order.begin(), order.end(), m.e) - order.begin()]);
                    ok = r.e == m.e && r.I == I && r.J == J && r.blk == blk;
                    mseen[blk] = 1;
                    ++covered;
                }
            if (!ok) {
                std::printf("FAIL macro S=%ld Sm=%ld item=%ld e=%d P=%d Q=%d\n", (long)S, (long)Sm, (long)it, m.e, m.P,
                            m.Q);
                return 1;
            }
        }
        if (covered != nblocks) {
            std::printf("FAIL macro S=%ld Sm=%ld covered %ld of %ld\n", (long)S, (long)Sm, (long)covered,
                        (long)nblocks);
            return 1;
        }
    }
    return 0;
}

// The 2-D grid of the per-item launches: every dimension stays under 2^32
// work-items (1024 per workgroup at most), rows of workgroups are a multiple
// of 8 whenever there is more than one, the grid holds every logical
// workgroup, and the XCD-aware map of the linear index onto items is one to
// one over the logical workgroups.
static int check_grid(int64_t blocks) {
    const dim3 g = grid_2d(blocks);
    const int64_t gx = g.x, gy = g.y;
    if (gx < 1 || gx > GRID_ROW || gx * 1024 >= (1ll << 32) || gy * 1024 >= (1ll << 32) || gx * gy < blocks ||
        gx * (gy - 1) >= blocks || (gy > 1 && (gx % 8 || gx * gy - blocks >= 8 * gy))) {
        std::printf("FAIL grid blocks=%ld gx=%ld gy=%ld\n", (long)blocks, (long)gx, (long)gy);
        return 1;
    }
    if (blocks % 8 == 0 && blocks <= 3000000) {
        const int64_t per = blocks / 8;
        std::vector<char> hit((size_t)blocks, 0);
        for (int64_t bl = 0; bl < blocks; ++bl) {
            const int64_t item = (bl % 8) * per + bl / 8;
            if (item < 0 || item >= blocks || hit[item]++) {
                std::printf("FAIL xcd map blocks=%ld bl=%ld\n", (long)blocks, (long)bl);
                return 1;
            }
        }
    }
    return 0;
}

int main(int argc, char **argv) {
    for (int64_t blocks : {1ll, 7ll, 8ll, 65535ll, 65536ll, 65537ll, 65544ll, 89375ll, 131071ll, 2950000ll,
                           5206528ll, 8906040ll, 1ll << 31})
        if (check_grid(blocks)) return 1;
    const int64_t tmax = argc > 1 ? std::atoll(argv[1]) : 200;
    std::set<int64_t> sizes = {1, 5, 8, 24};
    for (int prec = 0; prec < 5; ++prec)
        for (int d : {1, 32, 64, 200, 256, 257, 512, 2050}) sizes.insert(supertile_size(d) + 0 * prec);
    int64_t items = 0;
    for (int64_t S : sizes)
        for (int64_t t = 1; t <= tmax; ++t)
            if (check(S, {t / 2 + 1, 0, t, (t * 7) % 13}, items)) return 1;
    std::printf("ok %ld\n", (long)items);
    return 0;
}
