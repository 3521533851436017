"""GPU mapper vs the FP64 oracle, through the C ABI (needs an MI355X).

The graph (node elements, node CSR, edges, weights) must be bit-identical to
the oracle's for every tile precision; with the debug flag the per-stage
arrays (lens values, cover endpoints, pullback sets, neighbour counts, core
flags, node labels) must be identical too.  Sizes are chosen so that the
oracle finishes in seconds while cover elements still span several 128-row
tiles with ragged tails.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03209_amd import synth

pytestmark = pytest.mark.gpu

PRECS = [synth.PREC_FP32, synth.PREC_BF16, synth.PREC_BF16X3, synth.PREC_FP16,
         synth.PREC_FP16X3, synth.PREC_AUTO]


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_03209_amd import binding
    c = binding.Context(arena_bytes=48 << 30)
    yield c
    c.close()


def same_graph(g, ref):
    assert g.n_nodes == ref.n_nodes, (g.n_nodes, ref.n_nodes)
    assert np.array_equal(g.node_element, ref.node_element)
    assert np.array_equal(g.node_offsets, ref.node_offsets)
    assert np.array_equal(g.node_members, ref.node_members)
    assert np.array_equal(g.edges, ref.edges)
    assert np.array_equal(g.edge_weights, ref.edge_weights)


def same_stages(g, ref, n_axes):
    s = g.stages
    assert s["lens"].view(np.uint64).tolist() == ref.lens.reshape(-1).view(np.uint64).tolist()
    assert np.array_equal(s["lo"], np.concatenate(ref.lo))
    assert np.array_equal(s["hi"], np.concatenate(ref.hi))
    assert np.array_equal(s["elem_offsets"], ref.elem_offsets)
    assert np.array_equal(s["elem_members"], ref.elem_members)
    assert np.array_equal(s["slot_count"], ref.slot_count)
    assert np.array_equal(s["slot_core"].astype(bool), ref.slot_core.astype(bool))
    assert np.array_equal(s["slot_node"], ref.slot_node)


_ORACLE = {}


def oracle_graph(X, params):
    """The oracle does not depend on the tile precision: cache it per input."""
    key = (X.shape, float(np.float64(X).sum()), float(np.abs(np.float64(X)).sum()), params.eps,
           params.min_pts, tuple((a.kind, a.column, a.n_intervals, a.overlap, getattr(a, "cover", 0),
                                  None if a.direction is None else a.direction.tobytes(),
                                  None if a.values is None else a.values.tobytes()) for a in params.axes))
    if key not in _ORACLE:
        _ORACLE[key] = O.mapper(X, params)
    return _ORACLE[key]


def run_and_compare(ctx, X, params, stages=True):
    print(f"[case] n={X.shape[0]} d={X.shape[1]} prec={params.precision}", flush=True)
    cloud = ctx.cloud(X)
    try:
        g = cloud.run(params, debug=stages)
    finally:
        cloud.destroy()
    ref = oracle_graph(X, params)
    if stages:
        same_stages(g, ref, len(params.axes))
    same_graph(g, ref)
    # the run's reservation (taken after binning) held every later array,
    # unless the band list had to grow
    assert g.stats["reserved_bytes"] > 0
    assert g.stats["reserve_overflow_bytes"] == 0 or g.stats["tile_launches"] > 1
    return g, ref


def with_prec(params, prec):
    import copy
    p = copy.copy(params)
    p.precision = prec
    return p


@pytest.mark.parametrize("prec", PRECS)
def test_circle(ctx, prec):
    w = synth.circle_2k()
    g, ref = run_and_compare(ctx, w.X, with_prec(w.params, prec))
    assert g.n_nodes == 18 and g.n_edges == 18


@pytest.mark.parametrize("prec", PRECS)
def test_elements_across_supertiles(ctx, prec):
    """Two elements of 40-60 tile rows each, so the tile pairs of one element
    span several supertile columns (24 x 24 for the hi/lo splits, 8 x 8
    otherwise), the last one partial, with a ragged last tile: the tile order,
    the bitmask block numbering and the components' block lookups are all
    exercised off the diagonal supertiles, and the whole graph and every stage
    are compared with the oracle."""
    rng = np.random.default_rng(20110327)
    X, _ = synth.gaussian_mixture(rng, 9001, 48, 12)
    params = synth.Params([synth.Axis(synth.LENS_PROJECTION, 2, 0.4, direction=synth.unit_vector(rng, 48))],
                          eps=10.0, min_pts=8, precision=prec)
    g, ref = run_and_compare(ctx, X, params)
    sizes = np.diff(ref.elem_offsets)
    assert sizes.max() > 24 * 128 and sizes.min() > 8 * 128, sizes
    assert all(s % 128 for s in sizes), sizes
    assert g.n_nodes > 2


def _sized_elements(sizes, d, seed):
    """A mixture cloud whose cover elements have exactly the given sizes: the
    lens is the group index (VALUES), one interval per group, no overlap."""
    rng = np.random.default_rng(seed)
    X, _ = synth.gaussian_mixture(rng, int(sum(sizes)), d, 6)
    f = np.repeat(np.arange(len(sizes), dtype=np.float64), sizes)
    f = f[rng.permutation(f.shape[0])]
    params = synth.Params([synth.Axis(synth.LENS_VALUES, len(sizes), 0.0, values=f)],
                          eps=1.05 * float(np.sqrt(2.0 * d)), min_pts=6)
    return X, params


@pytest.mark.parametrize("prec", [synth.PREC_FP16, synth.PREC_BF16])
@pytest.mark.parametrize("d", [72, 256])
def test_macro_tiles(ctx, prec, d):
    """Macro tiles (pairs of 256-row blocks, up to four tile pairs per
    workgroup) against the oracle and against the tile-pair form: elements
    of one partial tile, of two tiles (one diagonal macro tile holding a
    diagonal, an off-diagonal and an absent tile pair), odd tile counts (a
    last macro row of one tile row), and enough macro rows to span several
    4 x 4 macro supertile columns, all with ragged tails."""
    from paper_2011_03209_amd import binding
    sizes = [50, 200, 130, 657, 1100, 3033]
    X, params = _sized_elements(sizes, d, 20110 + d)
    params = with_prec(params, prec)
    g, ref = run_and_compare(ctx, X, params)
    assert np.array_equal(np.diff(ref.elem_offsets), sizes)
    cloud = ctx.cloud(X)
    try:
        gp = cloud.run(params, debug=True, flags=binding.FLAG_TILE_PAIRS)
        gm = cloud.run(params, debug=True, flags=binding.FLAG_TILE_MACRO)
    finally:
        cloud.destroy()
    assert gp.stats["tile_m"] == 128 and gm.stats["tile_m"] == 256
    assert gm.stats["tiles_screened_out"] == 0
    # the same tile pairs computed in the same order: the same band pairs
    # (the default run screens tile pairs out, so it may have fewer)
    if gp.stats["tiles_screened_out"] == 0:
        assert gp.stats["band_pairs"] == gm.stats["band_pairs"]
    assert g.stats["band_pairs"] <= gm.stats["band_pairs"]
    for k in ("slot_count", "slot_core", "slot_node"):
        assert np.array_equal(gp.stages[k], gm.stages[k]), k
    same_graph(gp, ref)
    same_graph(gm, ref)


@pytest.mark.parametrize("prec", [synth.PREC_FP32, synth.PREC_BF16X3, synth.PREC_FP16])
def test_screening_exact_at_eps(ctx, prec):
    """Tile pairs are skipped only when their cells' balls prove them empty.
    Groups of 300 identical points (four cells, balls of radius 0) on the
    first axis at 0, 2,
    4 + 2^-20 and 100 with eps = 2: the first two are exactly eps apart
    (D = eps^2, neighbours, one cluster), the third lies just beyond eps of
    the second (its own cluster), the fourth is far (its tile pairs are
    screened out).  The graph is the oracle's and the unscreened one's."""
    from paper_2011_03209_amd import binding
    d = 16
    X = np.zeros((1200, d), np.float32)
    for g, x0 in enumerate((0.0, 2.0, 4.0 + 2.0 ** -20, 100.0)):
        X[300 * g:300 * (g + 1), 0] = x0
    X = X[np.random.default_rng(5).permutation(1200)]
    params = synth.Params([synth.Axis(synth.LENS_COLUMN, 1, 0.0, column=1)], eps=2.0, min_pts=5, precision=prec)
    g, ref = run_and_compare(ctx, X, params)
    assert g.n_nodes == 3, g.n_nodes
    assert g.stats["tiles_screened_out"] > 0
    cloud = ctx.cloud(X)
    try:
        gn = cloud.run(params, flags=binding.FLAG_NO_SCREEN)
    finally:
        cloud.destroy()
    assert gn.stats["tiles_screened_out"] == 0
    same_graph(gn, ref)


def test_screening_on_blobs(ctx):
    """Well separated blobs (R^32, 4 blobs 40 sigma apart, 20,000 points, one
    interval): most tile pairs join two blobs and are screened out (tiles
    that straddle two blobs in the locality order are kept); the graph is
    the oracle's."""
    rng = np.random.default_rng(31)
    X, _ = synth.blobs(rng, 20000, 32, 4, 40.0)
    params = synth.Params([synth.Axis(synth.LENS_L2, 1, 0.0)], eps=9.0, min_pts=6, precision=synth.PREC_BF16X3)
    g, ref = run_and_compare(ctx, X, params)
    assert g.stats["tiles_screened_out"] > g.stats["tiles"], (g.stats["tiles_screened_out"], g.stats["tiles"])
    assert g.stats["pairs_computed"] < g.stats["pairs"]


def test_screening_far_outliers(ctx):
    """Blobs with a 30% uniform background and a bridge of points between
    two blobs: the background lies outside every landmark cell (the outlier
    cell), and each such point farther than eps from every landmark cell's
    ball is screened against the cells (it can only neighbour other
    outliers); bridge points within eps of a blob are not.  The graph is the
    oracle's and the unscreened run's; most tile pairs are screened out,
    which the background rows would prevent if outliers stayed near every
    cell."""
    from paper_2011_03209_amd import binding
    rng = np.random.default_rng(47)
    Xb, _ = synth.blobs(rng, 14000, 32, 4, 40.0)
    lo, hi = Xb.min(axis=0), Xb.max(axis=0)
    bg = (lo + rng.uniform(0.0, 1.0, size=(6000, 32)) * (hi - lo)).astype(np.float32)
    t = np.linspace(0.0, 1.0, 60)[:, None]
    c0 = np.zeros(32); c1 = np.zeros(32)
    c0[0] = 40.0; c1[1] = 40.0
    bridge = (c0 + t * (c1 - c0) + rng.normal(0.0, 0.05, size=(60, 32))).astype(np.float32)
    X = np.ascontiguousarray(np.concatenate([Xb, bg, bridge])[rng.permutation(20060)])
    params = synth.Params([synth.Axis(synth.LENS_L2, 1, 0.0)], eps=9.0, min_pts=6, precision=synth.PREC_BF16X3)
    g, ref = run_and_compare(ctx, X, params)
    assert g.stats["tiles_screened_out"] > g.stats["tiles"], (g.stats["tiles_screened_out"], g.stats["tiles"])
    cloud = ctx.cloud(X)
    try:
        gn = cloud.run(params, flags=binding.FLAG_NO_SCREEN)
    finally:
        cloud.destroy()
    assert gn.stats["tiles_screened_out"] == 0
    same_graph(gn, ref)


def test_autotuner_measures_then_caches():
    """MAPPER_PREC_AUTO on the first run of its kind times every precision on
    a sample of the run's own tile pairs and picks the smallest predicted
    time; the next run of the same kind reuses the choice without sampling.
    Both graphs are the oracle's."""
    from paper_2011_03209_amd import binding
    w = synth.mixture_1m_d256(scale=0.03)
    params = with_prec(w.params, synth.PREC_AUTO)
    c = binding.Context(arena_bytes=8 << 30)
    try:
        cloud = c.cloud(w.X)
        g1 = cloud.run(params, debug=True)
        g2 = cloud.run(params)
        cloud.destroy()
    finally:
        c.close()
    pred = g1.stats["tune_pred_ms"]
    assert g1.stats["tune_sampled"] == 1 and all(t > 0 for t in pred), pred
    assert g1.stats["precision"] == int(np.argmin(pred)), (g1.stats["precision"], pred)
    assert g2.stats["tune_sampled"] == 0 and g2.stats["precision"] == g1.stats["precision"]
    ref = oracle_graph(w.X, params)
    same_stages(g1, ref, 1)
    same_graph(g1, ref)
    same_graph(g2, ref)


@pytest.mark.parametrize("prec", PRECS)
def test_mixture_d64(ctx, prec):
    w = synth.mixture_100k_d64(scale=0.06)
    g, _ = run_and_compare(ctx, w.X, with_prec(w.params, prec))
    assert g.stats["band_pairs"] >= 0


@pytest.mark.parametrize("prec", PRECS)
def test_mixture_d256(ctx, prec):
    w = synth.mixture_1m_d256(scale=0.012)
    g, _ = run_and_compare(ctx, w.X, with_prec(w.params, prec))
    assert g.stats["pairs"] > 0


@pytest.mark.parametrize("prec", [synth.PREC_FP32, synth.PREC_FP16X3, synth.PREC_BF16])
def test_grid_2d(ctx, prec):
    w = synth.mixture_500k_d128_2d(scale=0.012)
    run_and_compare(ctx, w.X, with_prec(w.params, prec))


def _cases():
    rng = np.random.default_rng(77)
    out = []
    # one point
    out.append(("one_point", np.array([[1.0, 2.0]], np.float32),
                synth.Params([synth.Axis(synth.LENS_COLUMN, 3, 0.2, column=0)], 0.5, 1)))
    # all points identical: degenerate lens range, every point in every interval
    out.append(("identical", np.ones((300, 5), np.float32),
                synth.Params([synth.Axis(synth.LENS_L2, 4, 0.25)], 0.0, 3)))
    # eps = 0: only duplicates are neighbours
    Xd = rng.integers(0, 3, size=(400, 2)).astype(np.float32)
    out.append(("eps0_duplicates", Xd, synth.Params([synth.Axis(synth.LENS_COLUMN, 2, 0.5, column=0)], 0.0, 2)))
    # minPts = 1, single interval, d = 1
    X1 = np.sort(rng.uniform(0, 100, size=(700, 1)).astype(np.float32), axis=0)
    out.append(("d1_minpts1", X1, synth.Params([synth.Axis(synth.LENS_COLUMN, 1, 0.0, column=0)], 0.3, 1)))
    # ragged K (d = 300) with element sizes around tile boundaries
    for n in (127, 128, 129, 255, 257):
        X = rng.normal(size=(n, 300)).astype(np.float32)
        out.append((f"d300_n{n}", X, synth.Params([synth.Axis(synth.LENS_LINF, 1, 0.0)], 24.4, 3)))
    # empty intervals (a gap in the lens), values lens, many intervals
    Xg = np.concatenate([rng.normal(0, 1, (300, 3)), rng.normal(40, 1, (300, 3))]).astype(np.float32)
    out.append(("gap", Xg, synth.Params([synth.Axis(synth.LENS_COLUMN, 25, 0.3, column=0)], 1.2, 4)))
    vals = rng.normal(size=500)
    Xv = rng.normal(size=(500, 7)).astype(np.float32)
    out.append(("values", Xv, synth.Params([synth.Axis(synth.LENS_VALUES, 6, 0.45, values=vals)], 3.0, 4)))
    out.append(("many_intervals", Xv, synth.Params([synth.Axis(synth.LENS_VALUES, 300, 0.6, values=vals)], 3.0, 2)))
    # overlap >= 1/2: non-adjacent intervals share points
    out.append(("overlap_0.8", Xv, synth.Params([synth.Axis(synth.LENS_L2, 7, 0.8)], 2.5, 3)))
    # huge offset: large norms, cancellation in the Gram form
    Xo = (rng.normal(size=(600, 64)) + 1000.0).astype(np.float32)
    out.append(("offset1000", Xo, synth.Params([synth.Axis(synth.LENS_L2, 5, 0.3)], 11.3, 5)))
    # tiny magnitudes (power-of-two rescaling keeps FP32/FP16 tiles exact-safe)
    Xs = (rng.normal(size=(500, 16)) * 1e-20).astype(np.float32)
    out.append(("tiny", Xs, synth.Params([synth.Axis(synth.LENS_L2, 3, 0.3)], 5.5e-20, 4)))
    # huge magnitudes (FP64 distances far above FP32 range after scaling back)
    Xh = (rng.normal(size=(400, 24)) * 1e30).astype(np.float32)
    out.append(("huge", Xh, synth.Params([synth.Axis(synth.LENS_L2, 4, 0.3)], 6.0e30, 4)))
    # very wide rows: many stages, ragged last one
    Xw = rng.normal(size=(200, 2050)).astype(np.float32)
    out.append(("d2050", Xw, synth.Params([synth.Axis(synth.LENS_LINF, 2, 0.3)], 64.0, 3)))
    # one 128-row block with 40 non-core rows, each within eps of cores of
    # two clusters: lines of cores at x = 0 and x = 10 (y = 0 .. 120), border
    # points at (5, 3k + 0.5) with 7 neighbours (minPts 8), listed first so
    # they share row block 0; each joins the lower cluster id (R3)
    ya = np.arange(121, dtype=np.float32)
    Xa = np.stack([np.zeros(121, np.float32), ya], axis=1)
    Xb2 = np.stack([np.full(121, 10.0, np.float32), ya], axis=1)
    Xbd = np.stack([np.full(40, 5.0, np.float32), 3.0 * np.arange(40, dtype=np.float32) + 0.5], axis=1)
    out.append(("border_two_clusters", np.ascontiguousarray(np.concatenate([Xbd, Xa, Xb2])),
                synth.Params([synth.Axis(synth.LENS_COLUMN, 1, 0.0, column=1)], 5.05, 8)))
    # 2-D with one axis of one interval
    out.append(("2d_1x9", Xv, synth.Params([synth.Axis(synth.LENS_COLUMN, 1, 0.0, column=0),
                                             synth.Axis(synth.LENS_COLUMN, 9, 0.5, column=1)], 3.0, 3)))
    return out


CASES = _cases()


@pytest.mark.parametrize("prec", [synth.PREC_FP32, synth.PREC_BF16X3, synth.PREC_FP16])
@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_edge_cases(ctx, case, prec):
    name, X, params = CASES[case]
    run_and_compare(ctx, X, with_prec(params, prec))


@pytest.mark.parametrize("case", range(len(CASES)), ids=[c[0] for c in CASES])
def test_edge_cases_eps_sweep(ctx, case):
    """The eps sweep on every edge case: eps, half of it and twice it in one
    pass, each graph the oracle's."""
    import copy
    name, X, params = CASES[case]
    params = with_prec(params, synth.PREC_BF16X3)
    eps = [params.eps, params.eps * 0.5, params.eps * 2.0]
    cloud = ctx.cloud(X)
    try:
        gs = cloud.run_eps_sweep(params, eps, debug=True)
    finally:
        cloud.destroy()
    for e, g in zip(eps, gs):
        p = copy.copy(params)
        p.eps = e
        ref = oracle_graph(X, p)
        same_stages(g, ref, len(p.axes))
        same_graph(g, ref)


@pytest.mark.parametrize("seed", range(4))
def test_dyadic_ties(ctx, seed):
    """Exact ties D == eps^2 and f == endpoint (the oracle is pinned to exact
    arithmetic on these inputs)."""
    rng = np.random.default_rng(500 + seed)
    X = synth.dyadic_cloud(rng, 900, 3, grid=4, span=12)
    params = synth.Params([synth.Axis(synth.LENS_COLUMN, 3, 0.5, column=0)], eps=0.75, min_pts=4,
                          precision=[synth.PREC_FP32, synth.PREC_BF16, synth.PREC_FP16X3, synth.PREC_BF16X3][seed])
    g, ref = run_and_compare(ctx, X, params)
    assert g.stats["band_pairs"] > 0          # ties must have gone through the FP64 recheck


def _d64(X, rows):
    return O.all_d2(X, rows)


@pytest.mark.parametrize("prec", [synth.PREC_FP32, synth.PREC_BF16, synth.PREC_BF16X3,
                                  synth.PREC_FP16, synth.PREC_FP16X3])
@pytest.mark.parametrize("data", ["mix256", "offset", "neardup"])
def test_tile_distances(ctx, prec, data):
    """FP32 tiles: |D_tile - D64| <= 1e-5 (|x|^2 + |y|^2).  Every precision:
    |D_tile - D64| <= the certified band the tile uses for its decisions."""
    rng = np.random.default_rng(9)
    if data == "mix256":
        X, _ = synth.gaussian_mixture(rng, 300, 256, 4)
    elif data == "offset":
        X = (rng.normal(size=(300, 96)) + 3000.0).astype(np.float32)
    else:
        base = rng.normal(size=(30, 128)).astype(np.float32)
        X = np.repeat(base, 10, axis=0) + rng.normal(scale=1e-4, size=(300, 128)).astype(np.float32)
        X = X.astype(np.float32)
    cloud = ctx.cloud(X)
    try:
        rows = np.arange(X.shape[0], dtype=np.int32)
        d2, band = cloud.tile_d2(rows, prec, eps=1.0)
    finally:
        cloud.destroy()
    ref = _d64(X, rows)
    nrm = (X.astype(np.float64) ** 2).sum(axis=1)
    err = np.abs(d2 - ref)
    assert np.all(err <= band), float((err - band).max())
    if prec == synth.PREC_FP32:
        assert np.all(err <= 1e-5 * (nrm[:, None] + nrm[None, :]))


@pytest.fixture(scope="module")
def large_cloud():
    """10,000 points of a 256-D mixture with a large common offset on a
    quarter of them (large |x|), and their exact pairwise distances."""
    rng = np.random.default_rng(21)
    X, _ = synth.gaussian_mixture(rng, 10_000, 256, 12)
    X[:2500] += np.float32(40.0)
    X = np.ascontiguousarray(X, dtype=np.float32)
    rows = np.arange(X.shape[0], dtype=np.int32)
    return X, rows, _d64(X, rows)


@pytest.mark.parametrize("prec", [synth.PREC_FP32, synth.PREC_BF16, synth.PREC_BF16X3,
                                  synth.PREC_FP16, synth.PREC_FP16X3])
def test_tile_band_soundness_1e8_pairs(ctx, large_cloud, prec):
    """Band soundness on 1e8 ordered pairs per precision: every tile distance
    lies within its certified band of the exact FP64 distance."""
    X, rows, ref = large_cloud
    cloud = ctx.cloud(X)
    try:
        d2, band = cloud.tile_d2(rows, prec, eps=20.0)
    finally:
        cloud.destroy()
    assert d2.shape == ref.shape == (10_000, 10_000)
    over = np.abs(d2 - ref) - band
    assert float(over.max()) <= 0.0, float(over.max())


@pytest.mark.parametrize("prec", [synth.PREC_FP32, synth.PREC_BF16, synth.PREC_BF16X3,
                                  synth.PREC_FP16, synth.PREC_FP16X3])
@pytest.mark.parametrize("load", ["grid2d_d128", "d256", "d40"])
def test_precisions_match_oracle(ctx, prec, load):
    """Every tile precision gives the oracle's graph: ragged elements, 2-D
    covers, widths that are and are not multiples of a stage."""
    if load == "grid2d_d128":
        w = synth.mixture_500k_d128_2d(scale=0.01, precision=prec)
    elif load == "d256":
        w = synth.mixture_1m_d256(scale=0.004, precision=prec)
    else:
        w = synth.mixture_100k_d64(scale=0.05)
        w.X = np.ascontiguousarray(w.X[:, :40])
        w.params.precision = prec
    cloud = ctx.cloud(w.X)
    try:
        g = cloud.run(w.params)
    finally:
        cloud.destroy()
    same_graph(g, oracle_graph(w.X, w.params))


def test_band_list_regrows(ctx):
    """Plain BF16 on one 35k-point element leaves tens of band pairs per tile,
    more than the first band list holds: the list grows, the tiles are redone,
    and the graph is still the oracle's."""
    w = synth.mixture_1m_d256(scale=0.035, precision=synth.PREC_BF16)
    ax = w.params.axes[0]
    params = synth.Params([synth.Axis(ax.kind, 1, 0.0, direction=ax.direction)], eps=w.params.eps,
                          min_pts=w.params.min_pts, precision=synth.PREC_BF16)
    cloud = ctx.cloud(w.X)
    try:
        g = cloud.run(params)
    finally:
        cloud.destroy()
    assert g.stats["tile_launches"] > 1, g.stats
    assert g.stats["band_pairs"] > 16 * g.stats["tiles"], g.stats
    assert g.stats["ms_recheck"] > 0 and g.stats["ms_tiles"] > 0 and g.stats["ms_cc"] > 0, g.stats
    same_graph(g, oracle_graph(w.X, params))


@pytest.mark.parametrize("n_pairs", [1023, 1024, 1025, 2047, 2048, 2049])
def test_sort_and_scan_sizes(ctx, n_pairs):
    """Well-separated pairs of points in one interval, minPts 2: every pair is
    a node, so the root sort sees n_pairs keys and the membership sorts and
    scans 2 n_pairs, on both sides of 2048, the largest count that one
    workgroup sorts or scans alone."""
    rng = np.random.default_rng(n_pairs)
    centers = rng.permutation(np.arange(4 * n_pairs))[:n_pairs, None] * np.ones((1, 8)) * 10.0
    centers[:, 1:] += rng.normal(scale=0.01, size=(n_pairs, 7))
    X = np.concatenate([centers + 0.1, centers - 0.1]).astype(np.float32)
    params = synth.Params([synth.Axis(synth.LENS_COLUMN, 1, 0.0, column=0)], eps=1.0, min_pts=2,
                          precision=synth.PREC_BF16X3)
    g, ref = run_and_compare(ctx, X, params)
    assert g.n_nodes == n_pairs


@pytest.mark.parametrize("case", ["mix1d", "grid2d_one_axis", "ties", "fewer_points_than_intervals"])
def test_balanced_cover(ctx, case):
    """The balanced cover (intervals holding equal numbers of points): the
    GPU's endpoints (from a device radix sort of the lens), elements, counts
    and graph equal the oracle's."""
    if case == "mix1d":
        w = synth.mixture_100k_d64(scale=0.05)
        w.params.axes[0].cover = 1
        X, params = w.X, with_prec(w.params, synth.PREC_BF16X3)
    elif case == "grid2d_one_axis":
        w = synth.mixture_500k_d128_2d(scale=0.01, precision=synth.PREC_FP16)
        w.params.axes[0].cover = 1
        X, params = w.X, w.params
    elif case == "ties":
        rng = np.random.default_rng(11)
        X = rng.normal(size=(6000, 16)).astype(np.float32)
        vals = np.floor(rng.uniform(0, 9, size=6000))               # nine distinct lens values
        params = synth.Params([synth.Axis(4, 7, 0.4, values=vals, cover=1)], eps=4.5, min_pts=5,
                              precision=synth.PREC_FP32)
    else:
        X = np.random.default_rng(5).normal(size=(5, 3)).astype(np.float32)
        params = synth.Params([synth.Axis(1, 8, 0.1, cover=1)], eps=2.0, min_pts=1,
                              precision=synth.PREC_FP32)
    run_and_compare(ctx, X, params)


@pytest.mark.parametrize("case", ["d64_fp32", "d256_bf16x3", "grid2d_fp16", "bf16_close_eps"])
def test_eps_sweep(ctx, case):
    """One pass for several eps values (any order, repeats allowed) gives for
    each value the oracle's graph and stages (counts, core flags, node of
    every slot); close values share band pairs, each re-decided per value."""
    import copy
    if case == "d64_fp32":
        w = synth.mixture_100k_d64(scale=0.05)
        params, eps = with_prec(w.params, synth.PREC_FP32), [12.5, 9.0, 15.0, 12.5]
    elif case == "d256_bf16x3":
        w = synth.mixture_1m_d256(scale=0.004, precision=synth.PREC_BF16X3)
        params, eps = w.params, [24.0, 22.6, 25.5]
    elif case == "grid2d_fp16":
        w = synth.mixture_500k_d128_2d(scale=0.01, precision=synth.PREC_FP16)
        params, eps = w.params, [17.0, 15.0, 19.0, 21.0]
    else:
        w = synth.mixture_1m_d256(scale=0.004, precision=synth.PREC_BF16)
        params, eps = w.params, [24.0, 24.01]
    print(f"[case] eps sweep {case} {eps}", flush=True)
    cloud = ctx.cloud(w.X)
    try:
        gs = cloud.run_eps_sweep(params, eps, debug=True)
        single = cloud.run(copy.copy(params), debug=False)
    finally:
        cloud.destroy()
    assert len(gs) == len(eps)
    for e, g in zip(eps, gs):
        p = copy.copy(params)
        p.eps = e
        ref = oracle_graph(w.X, p)
        same_stages(g, ref, len(p.axes))
        same_graph(g, ref)
    same_graph(single, gs[0])


def test_eps_sweep_errors(ctx):
    from paper_2011_03209_amd import binding
    w = synth.mixture_100k_d64(scale=0.01)
    cloud = ctx.cloud(w.X)
    try:
        for bad in ([], [1.0] * (binding.MAX_EPS_VALUES + 1), [1.0, -2.0], [float("nan")]):
            with pytest.raises(binding.MapperError):
                cloud.run_eps_sweep(w.params, bad)
        g = cloud.run_eps_sweep(w.params, [w.params.eps])[0]      # one value: the plain run
        same_graph(g, cloud.run(w.params))
    finally:
        cloud.destroy()


@pytest.mark.parametrize("case", ["d256_bf16x3", "grid2d_fp16x3"])
def test_eps_minpts_sweep(ctx, case):
    """One pass for every (eps, minPts) pair gives for each the oracle's
    graph and stages: minPts 1 (every point a core), the workload's own, and
    values that leave few or no cores; eps repeated and out of order."""
    import copy
    if case == "d256_bf16x3":
        w = synth.mixture_1m_d256(scale=0.004, precision=synth.PREC_BF16X3)
        eps, mps = [24.0, 22.6, 24.0], [10, 1, 40, 3]
    else:
        w = synth.mixture_500k_d128_2d(scale=0.01, precision=synth.PREC_FP16X3)
        eps, mps = [17.0, 19.0], [8, 2, 25]
    print(f"[case] eps x minPts sweep {case} {eps} {mps}", flush=True)
    cloud = ctx.cloud(w.X)
    try:
        gs = cloud.run_sweep(w.params, eps, mps, debug=True)
    finally:
        cloud.destroy()
    assert len(gs) == len(eps) and all(len(row) == len(mps) for row in gs)
    for e, row in zip(eps, gs):
        for m, g in zip(mps, row):
            p = copy.copy(w.params)
            p.eps, p.min_pts = e, m
            ref = oracle_graph(w.X, p)
            same_stages(g, ref, len(p.axes))
            same_graph(g, ref)


def test_eps_minpts_sweep_errors(ctx):
    from paper_2011_03209_amd import binding
    w = synth.mixture_100k_d64(scale=0.01)
    cloud = ctx.cloud(w.X)
    try:
        for bad in ([], [5] * (binding.MAX_MINPTS_VALUES + 1), [5, 0], [-1]):
            with pytest.raises(binding.MapperError):
                cloud.run_sweep(w.params, [w.params.eps], bad)
        with pytest.raises(binding.MapperError):
            cloud.run_sweep(w.params, [], [5])
        g = cloud.run_sweep(w.params, [w.params.eps], [w.params.min_pts])[0][0]   # one pair: the plain run
        same_graph(g, cloud.run(w.params))
    finally:
        cloud.destroy()


def test_determinism_and_permutation(ctx):
    w = synth.mixture_1m_d256(scale=0.008, precision=synth.PREC_BF16X3)
    cloud = ctx.cloud(w.X)
    g1 = cloud.run(w.params)
    g2 = cloud.run(w.params)
    cloud.destroy()
    same_graph(g1, g2)
    perm = np.random.default_rng(3).permutation(w.X.shape[0])
    cloud = ctx.cloud(w.X[perm])
    gp = cloud.run(w.params)
    cloud.destroy()
    # same clusters as point sets after mapping indices back (ids are canonical per input order)
    def sets(g, mapping):
        o = g.node_offsets
        return sorted((int(g.node_element[v]), tuple(sorted(mapping[g.node_members[o[v]:o[v + 1]]].tolist())))
                      for v in range(g.n_nodes))
    assert sets(g1, np.arange(w.X.shape[0])) == sets(gp, perm)


def test_serving_alone_vs_mix():
    """Requests submitted together (overlapping on several streams) give the
    same graphs as each request alone."""
    from paper_2011_03209_amd import binding
    ctx = binding.Context(arena_bytes=8 << 30, serving_streams=3)
    try:
        clouds = [ctx.cloud(X) for X in synth.serving_clouds(scale=0.01)]
        raw = synth.serving_clouds(scale=0.01)
        reqs = synth.serving_requests(raw, 12, qps=0.0)
        alone = [clouds[c].run(p) for (_, c, p) in reqs]
        tickets = [clouds[c].submit(p) for (_, c, p) in reqs]
        mixed = [binding.wait(ctx, t) for t in tickets]
        for a, b in zip(alone, mixed):
            same_graph(a, b)
        # and the oracle agrees on a few of them
        for k in (0, 5, 11):
            _, c, p = reqs[k]
            same_graph(mixed[k], O.mapper(raw[c], p))
        for c in clouds:
            c.destroy()
    finally:
        ctx.close()


def test_serving_under_memory_pressure():
    """Serving with an arena that holds the clouds and about one and a half
    of the largest request's reservation, on three stream slots.  A request
    reserves its whole workspace in one block after binning, before its tile
    pass; one that cannot have it waits (and holds the queue) until memory is
    returned, so no tile pass is ever thrown away, and every graph is the
    graph of its solo run."""
    from paper_2011_03209_amd import binding
    raw = synth.serving_clouds(scale=0.02)
    reqs = synth.serving_requests(raw, 12, qps=0.0)
    big = binding.Context(arena_bytes=8 << 30)
    try:
        clouds = [big.cloud(X) for X in raw]
        cloud_bytes = big.memory()[0]                   # the resident clouds
        alone = [clouds[c].run(p) for (_, c, p) in reqs]
        res = sorted((g.stats["reserved_bytes"] for g in alone), reverse=True)
        assert all(g.stats["reserve_overflow_bytes"] == 0 for g in alone)
        for c in clouds:
            c.destroy()
    finally:
        big.close()
    # the largest requests first (they start together on the three slots),
    # with room beside the largest reservation for half of the second one
    # (plus what three requests keep from their lens and binning stages: the
    # lens values and the slot arrays, 8 bytes per point and 12 per slot)
    order = sorted(range(len(reqs)), key=lambda k: -alone[k].stats["reserved_bytes"])
    phase_a = max(8 * raw[c].shape[0] + 12 * alone[k].stats["n_slots"] + 4096 for k, (_, c, _) in enumerate(reqs))
    ctx = binding.Context(arena_bytes=int(cloud_bytes + res[0] + 0.5 * res[1] + 3 * phase_a) + (1 << 20),
                          serving_streams=3)
    try:
        clouds = [ctx.cloud(X) for X in raw]
        tickets = {k: clouds[reqs[k][1]].submit(reqs[k][2]) for k in order}
        mixed = [binding.wait(ctx, tickets[k]) for k in range(len(reqs))]
        for a, b in zip(alone, mixed):
            same_graph(a, b)
        assert all(g.stats["tile_passes_redone"] == 0 for g in mixed)
        assert sum(g.stats["admission_waits"] for g in mixed) > 0     # the arena did run short
        for c in clouds:
            c.destroy()
    finally:
        ctx.close()


def test_serving_large_request_among_a_stream_of_small_ones():
    """A large request submitted into a continuing stream of small ones, with
    an arena that holds the large request's reservation only when few small
    ones run: once it has waited, no new request starts before it has its
    reservation, so it finishes while the small ones keep arriving."""
    import threading
    import time
    from paper_2011_03209_amd import binding
    rng = np.random.default_rng(9)
    Xs, _ = synth.gaussian_mixture(rng, 3000, 32, 5)
    Xl, _ = synth.gaussian_mixture(rng, 60000, 64, 8)
    ps = synth.Params([synth.Axis(synth.LENS_L2, 5, 0.3)], eps=8.4, min_pts=5, precision=synth.PREC_BF16X3)
    pl = synth.Params([synth.Axis(synth.LENS_L2, 2, 0.3)], eps=11.9, min_pts=8, precision=synth.PREC_BF16X3)
    probe = binding.Context(arena_bytes=8 << 30)
    try:
        cs, cl = probe.cloud(Xs), probe.cloud(Xl)
        gs_alone, gl_alone = cs.run(ps), cl.run(pl)
        t0 = time.perf_counter()
        cl.run(pl)
        solo_s = time.perf_counter() - t0
        rs, rl = gs_alone.stats["reserved_bytes"], gl_alone.stats["reserved_bytes"]
        cs.destroy()
        cl.destroy()
    finally:
        probe.close()
    assert rl > 8 * rs
    # room for the large reservation beside one small one, not two
    ctx = binding.Context(arena_bytes=int(Xs.nbytes + Xl.nbytes + rl + 1.5 * rs) + (16 << 20), serving_streams=3)
    stop = threading.Event()
    small = []
    try:
        cs, cl = ctx.cloud(Xs), ctx.cloud(Xl)

        def feed():
            while not stop.is_set():
                small.append(cs.submit(ps))
                time.sleep(0.002)

        th = threading.Thread(target=feed)
        th.start()
        time.sleep(0.2)
        tl = cl.submit(pl)
        budget = 1.0 + 20 * solo_s
        gl = binding.wait(ctx, tl, timeout_us=int(budget * 1e6))   # raises if the large one starves
        stop.set()
        th.join()
        same_graph(gl, gl_alone)
        assert gl.stats["tile_passes_redone"] == 0
        for t in small:
            g = binding.wait(ctx, t)
            assert g.stats["tile_passes_redone"] == 0
        same_graph(g, gs_alone)
        cs.destroy()
        cl.destroy()
    finally:
        stop.set()
        ctx.close()


def test_serving_new_features():
    """Serving requests that use the balanced cover and the whole-cloud
    lenses, mixed with plain ones, give the graphs of their solo runs and the
    oracle's."""
    from paper_2011_03209_amd import binding
    ctx = binding.Context(arena_bytes=8 << 30, serving_streams=3)
    try:
        X = np.ascontiguousarray(synth.mixture_100k_d64(scale=0.02).X[:, :24])
        cloud = ctx.cloud(X)
        reqs = [synth.Params([synth.Axis(synth.LENS_L2, 6, 0.3, cover=1)], eps=6.5, min_pts=4),
                synth.Params([synth.Axis(synth.LENS_ECCENTRICITY, 5, 0.4)], eps=6.5, min_pts=4),
                synth.Params([synth.Axis(synth.LENS_KNN_DISTANCE, 4, 0.3, column=3)], eps=6.0, min_pts=3,
                             precision=synth.PREC_FP16),
                synth.Params([synth.Axis(synth.LENS_L2, 8, 0.25)], eps=6.5, min_pts=4)]
        alone = [cloud.run(p) for p in reqs]
        tickets = [cloud.submit(p) for p in reqs]
        mixed = [binding.wait(ctx, tk) for tk in tickets]
        for a, b, p in zip(alone, mixed, reqs):
            same_graph(a, b)
            same_graph(b, O.mapper(X, p))
        cloud.destroy()
    finally:
        ctx.close()


def test_launch_beyond_2_32_work_items(ctx):
    """One element of 540,000 points: 8.9M tile pairs, so the tile launch
    (512 work-items per tile pair) exceeds the 2^32 work-items one grid
    dimension can dispatch and runs as a 2-D grid.  With eps above the
    cloud's diameter every pair is a neighbour, so every tile pair must have
    run: each point's count is n, and the graph is one node of all points."""
    rng = np.random.default_rng(20110330)
    n = 540_000
    X = rng.uniform(-1.0, 1.0, size=(n, 4)).astype(np.float32)
    params = synth.Params([synth.Axis(synth.LENS_COLUMN, 1, 0.0, column=0)], eps=10.0, min_pts=2,
                          precision=synth.PREC_FP16)
    assert (-(-n // 128)) * (-(-n // 128) + 1) // 2 * 512 > 2 ** 32
    cloud = ctx.cloud(X)
    try:
        g = cloud.run(params, debug=True)
    finally:
        cloud.destroy()
    assert g.n_nodes == 1 and g.n_edges == 0
    assert np.array_equal(g.node_members, np.arange(n, dtype=np.int32))
    assert np.all(g.stages["slot_count"] == n)


def test_errors(ctx):
    from paper_2011_03209_amd import binding
    X = np.random.default_rng(1).normal(size=(100, 4)).astype(np.float32)
    cloud = ctx.cloud(X)
    bad = [synth.Params([synth.Axis(synth.LENS_COLUMN, 0, 0.2)], 1.0, 2),
           synth.Params([synth.Axis(synth.LENS_COLUMN, 3, 1.0)], 1.0, 2),
           synth.Params([synth.Axis(synth.LENS_COLUMN, 3, 0.2, column=4)], 1.0, 2),
           synth.Params([synth.Axis(synth.LENS_COLUMN, 3, 0.2)], -1.0, 2),
           synth.Params([synth.Axis(synth.LENS_COLUMN, 3, 0.2)], float("nan"), 2),
           synth.Params([synth.Axis(synth.LENS_COLUMN, 3, 0.2)], 1.0, 0),
           synth.Params([synth.Axis(synth.LENS_VALUES, 3, 0.2,
                                    values=np.r_[-1.5e308, 1.5e308, np.zeros(98)])], 1.0, 2)]
    for p in bad:
        with pytest.raises(binding.MapperError) as ei:
            cloud.run(p)
        assert ei.value.code == binding.MAPPER_EINVAL
    Xn = X.copy()
    Xn[5, 2] = np.nan
    with pytest.raises(binding.MapperError) as ei:
        ctx.cloud(Xn)
    assert ei.value.code == binding.MAPPER_EINVAL
    # busy cloud
    t = cloud.submit(synth.Params([synth.Axis(synth.LENS_L2, 3, 0.2)], 1.0, 2))
    try:
        cloud.destroy()
        destroyed_early = True
    except binding.MapperError as e:
        assert e.code == binding.MAPPER_EBUSY
        destroyed_early = False
    binding.wait(ctx, t)
    if not destroyed_early:
        cloud.destroy()
    # a tiny arena: ENOMEM, then the context still works
    small = binding.Context(arena_bytes=2 << 20)
    try:
        big = small.cloud(np.random.default_rng(2).normal(size=(4000, 64)).astype(np.float32))
        with pytest.raises(binding.MapperError) as ei:
            big.run(synth.Params([synth.Axis(synth.LENS_L2, 1, 0.0)], 100.0, 2))
        assert ei.value.code == binding.MAPPER_ENOMEM
        big.destroy()
        ok = small.cloud(X)
        ok.run(synth.Params([synth.Axis(synth.LENS_L2, 2, 0.2)], 2.0, 2))
        ok.destroy()
    finally:
        small.close()


def check_nerve(g):
    """Edges are exactly the node pairs that share points, weighted by the
    number of shared points (the nerve of the cover by clusters)."""
    o = g.node_offsets
    owner = {}
    for v in range(g.n_nodes):
        for p in g.node_members[o[v]:o[v + 1]].tolist():
            owner.setdefault(p, []).append(v)
    want = {}
    for vs in owner.values():
        for i in range(len(vs)):
            for j in range(i + 1, len(vs)):
                want[(vs[i], vs[j])] = want.get((vs[i], vs[j]), 0) + 1
    got = {(int(a), int(b)): int(c) for (a, b), c in zip(g.edges, g.edge_weights)}
    assert got == want


def check_small_elements(g, X, params, f, lo, hi, count=6):
    """The smallest non-empty elements: their members are exactly the points
    inside them (per axis, closed intervals), and their neighbour counts and
    clusters are the oracle's DBSCAN of those members."""
    eo = g.stages["elem_offsets"]
    sizes = np.diff(eo)
    shape = [a.n_intervals for a in params.axes]
    checked = 0
    for e in np.argsort(sizes, kind="stable"):
        if sizes[e] == 0:
            continue
        idx = np.unravel_index(int(e), shape)
        inside = np.ones(X.shape[0], bool)
        for a in range(len(shape)):
            inside &= (lo[a][idx[a]] <= f[a]) & (f[a] <= hi[a][idx[a]])
        mem = g.stages["elem_members"][eo[e]:eo[e + 1]]
        want = np.nonzero(inside)[0]
        assert np.array_equal(mem, want)
        cnt, core, cid = O.dbscan(X, want, params.eps, params.min_pts)
        assert np.array_equal(g.stages["slot_count"][eo[e]:eo[e + 1]], cnt)
        node = g.stages["slot_node"][eo[e]:eo[e + 1]]
        first = node[node >= 0].min() if (node >= 0).any() else 0
        assert np.array_equal(np.where(node >= 0, node - first, -1), cid)
        checked += 1
        if checked == count:
            break
    assert checked > 0


def test_full_size_1m_d256(ctx):
    """Paper-scale cloud (1,000,000 x 256) in the benchmark's launch
    configuration: the BF16 split path and the FP32 path give the identical
    graph; sampled lens values and whole small elements match the oracle; the
    graph satisfies the nerve invariants."""
    w = synth.mixture_1m_d256()
    cloud = ctx.cloud(w.X)
    try:
        gb = cloud.run(with_prec(w.params, synth.PREC_BF16X3), debug=True)
        gf = cloud.run(with_prec(w.params, synth.PREC_FP32))
    finally:
        cloud.destroy()
    same_graph(gb, gf)
    ax = w.params.axes[0]
    f = O.lens(w.X, ax)                                     # the oracle's own lens of all points
    assert np.array_equal(gb.stages["lens"], f)
    lo, hi = O.cover(float(f.min()), float(f.max()), ax.n_intervals, ax.overlap)
    assert np.array_equal(gb.stages["lo"], lo) and np.array_equal(gb.stages["hi"], hi)
    eo = gb.stages["elem_offsets"]
    sizes = np.diff(eo)
    for e in np.argsort(sizes)[:6]:
        if sizes[e] == 0:
            continue
        mem = gb.stages["elem_members"][eo[e]:eo[e + 1]]
        want = np.nonzero((lo[e] <= f) & (f <= hi[e]))[0]
        assert np.array_equal(mem, want)
        cnt, core, cid = O.dbscan(w.X, want, w.params.eps, w.params.min_pts)
        assert np.array_equal(gb.stages["slot_count"][eo[e]:eo[e + 1]], cnt)
        node = gb.stages["slot_node"][eo[e]:eo[e + 1]]
        first = node[node >= 0].min() if (node >= 0).any() else 0
        assert np.array_equal(np.where(node >= 0, node - first, -1), cid)
    check_nerve(gb)


def test_full_size_balanced_cover(ctx):
    """1M x 256 with the balanced cover: the GPU's endpoints (device radix
    sort of the lens) are the oracle's, computed from the oracle's own lens,
    and the smallest elements hold exactly the points inside them."""
    w = synth.mixture_1m_d256()
    w.params.axes[0].cover = 1
    cloud = ctx.cloud(w.X)
    try:
        g = cloud.run(w.params, debug=True)
    finally:
        cloud.destroy()
    ax = w.params.axes[0]
    f = O.lens(w.X, ax)
    lo, hi = O.cover_balanced(f, ax.n_intervals, ax.overlap)
    assert np.array_equal(g.stages["lo"], lo) and np.array_equal(g.stages["hi"], hi)
    eo = g.stages["elem_offsets"]
    sizes = np.diff(eo)
    assert sizes.max() - sizes.min() <= 3
    for e in (0, ax.n_intervals // 2, ax.n_intervals - 1):
        mem = g.stages["elem_members"][eo[e]:eo[e + 1]]
        assert np.array_equal(mem, np.nonzero((lo[e] <= f) & (f <= hi[e]))[0])


def test_full_size_eps_sweep(ctx):
    """1M x 256, the four eps values the benchmark sweeps: each graph of the
    one-pass sweep is the graph of its own run."""
    import copy
    w = synth.mixture_1m_d256()
    eps = [20.0, 22.0, 24.0, 26.0]
    cloud = ctx.cloud(w.X)
    try:
        gs = cloud.run_eps_sweep(w.params, eps)
        for e, g in zip(eps, gs):
            p = copy.copy(w.params)
            p.eps = e
            same_graph(g, cloud.run(p))
    finally:
        cloud.destroy()


def test_full_size_repeatable(ctx):
    """1M x 256 at eps = 20 (many small clusters, the most merging in the
    components pass), run eight times: every graph is the same.  Components
    are built with concurrent unions and path halving; the final labels must
    not depend on their timing."""
    import copy
    w = synth.mixture_1m_d256()
    p = copy.copy(w.params)
    p.eps = 20.0
    cloud = ctx.cloud(w.X)
    try:
        first = cloud.run(p)
        for _ in range(7):
            same_graph(cloud.run(p), first)
    finally:
        cloud.destroy()


def test_full_size_100k_d64(ctx):
    """The 100k x 64 configuration at full size: the whole graph and every
    stage are the oracle's, in the plain FP32 path and in the matrix-core
    precisions."""
    w = synth.mixture_100k_d64()
    for prec in (synth.PREC_FP32, synth.PREC_BF16X3, synth.PREC_FP16, synth.PREC_AUTO):
        g, ref = run_and_compare(ctx, w.X, with_prec(w.params, prec))
    assert g.n_nodes == ref.n_nodes > 20


def test_full_size_grid_500k_d128(ctx):
    """The 2-D configuration at full size (525,000 x 128, 15 x 15 cells, 225
    elements of uneven sizes): FP16 single products (about 3e8 band pairs
    re-decided in FP64), the FP16 split and the FP32 path give one graph; the
    lens values and endpoints of both axes are the oracle's; the smallest
    elements match the oracle's DBSCAN; the edges are the nerve."""
    w = synth.mixture_500k_d128_2d()
    cloud = ctx.cloud(w.X)
    try:
        g16 = cloud.run(with_prec(w.params, synth.PREC_FP16), debug=True)
        gx = cloud.run(with_prec(w.params, synth.PREC_FP16X3))
        gf = cloud.run(with_prec(w.params, synth.PREC_FP32))
    finally:
        cloud.destroy()
    same_graph(g16, gf)
    same_graph(gx, gf)
    assert g16.stats["band_pairs"] > 10 ** 7
    f = [O.lens(w.X, ax) for ax in w.params.axes]
    assert np.array_equal(g16.stages["lens"], np.concatenate(f))
    lo, hi = [], []
    for a, ax in enumerate(w.params.axes):
        l, h = O.cover(float(f[a].min()), float(f[a].max()), ax.n_intervals, ax.overlap)
        lo.append(l)
        hi.append(h)
    assert np.array_equal(g16.stages["lo"], np.concatenate(lo))
    assert np.array_equal(g16.stages["hi"], np.concatenate(hi))
    check_small_elements(g16, w.X, w.params, f, lo, hi)
    check_nerve(g16)


def test_full_size_serving():
    """The serving form at full size (the eight resident clouds of 10k to 500k
    points, the benchmark's stream slots): requests submitted together give
    the graphs of their solo runs, and the oracle agrees on the requests to
    the 10k-point clouds."""
    from paper_2011_03209_amd import binding, serve
    ctx = binding.Context(arena_bytes=64 << 30, serving_streams=serve.SLOTS)
    try:
        raw = synth.serving_clouds()
        clouds = [ctx.cloud(X) for X in raw]
        reqs = synth.serving_requests(raw, 10, qps=0.0)
        alone = [clouds[c].run(p) for (_, c, p) in reqs]
        tickets = [clouds[c].submit(p) for (_, c, p) in reqs]
        mixed = [binding.wait(ctx, t) for t in tickets]
        for a, b in zip(alone, mixed):
            same_graph(a, b)
        small = [k for k, (_, c, _) in enumerate(reqs) if raw[c].shape[0] <= 10_000]
        for k in small[:2]:
            _, c, p = reqs[k]
            same_graph(mixed[k], O.mapper(raw[c], p))
        assert len({c for (_, c, _) in reqs}) >= 4
        for c in clouds:
            c.destroy()
    finally:
        ctx.close()
