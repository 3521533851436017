"""Pins of the FP64 oracle against exact rational arithmetic (CPU only).

Dyadic inputs (multiples of 1/8, small magnitude) make every FP64 operation in
the oracle exact, so its lens values, cover endpoints, neighbour decisions --
ties D == eps^2 and f == endpoint included -- and the whole graph must equal
the exact mapper built from the definitions in tests/exact_mapper.py.
"""
from fractions import Fraction as F

import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03209_amd import synth
from tests import exact_mapper as EX


def _compare(X, params, exact_endpoints=True):
    g = O.mapper(X, params)
    if exact_endpoints:
        ref = EX.exact_mapper(X, params)
    else:
        eps_ = [([F(v) for v in g.lo[a]], [F(v) for v in g.hi[a]]) for a in range(len(params.axes))]
        ref = EX.exact_mapper(X, params, endpoints=eps_)
    for a in range(len(params.axes)):
        assert [F(v) for v in g.lens[a]] == ref["lens"][a]
        if exact_endpoints:
            assert [F(v) for v in g.lo[a]] == ref["lo"][a]
            assert [F(v) for v in g.hi[a]] == ref["hi"][a]
    eo = g.elem_offsets
    got_elems = [g.elem_members[eo[e]:eo[e + 1]].tolist() for e in range(len(eo) - 1)]
    assert got_elems == ref["elements"]
    assert g.slot_count.tolist() == ref["slot_count"]
    assert [bool(c) for c in g.slot_core] == ref["slot_core"]
    no = g.node_offsets
    got_nodes = [g.node_members[no[v]:no[v + 1]].tolist() for v in range(g.n_nodes)]
    assert got_nodes == ref["nodes"]
    assert g.node_element.tolist() == ref["node_elem"]
    got_edges = {(int(a), int(b)): int(w) for (a, b), w in zip(g.edges, g.edge_weights)}
    assert got_edges == ref["edges"]
    assert [tuple(e) for e in g.edges.tolist()] == sorted(ref["edges"].keys())
    return g, ref


# (n_intervals, overlap) pairs with n - (n-1)p a power of two, so the cover
# endpoints are exact in FP64 for dyadic ranges.
EXACT_COVERS = [(1, 0.0), (2, 0.0), (3, 0.5), (5, 0.25), (9, 0.875), (4, 0.0)]


@pytest.mark.parametrize("seed", range(12))
def test_dyadic_1d_exact(seed):
    rng = np.random.default_rng(1000 + seed)
    n = int(rng.integers(5, 36))
    d = int(rng.integers(1, 5))
    X = synth.dyadic_cloud(rng, n, d)
    nint, p = EXACT_COVERS[seed % len(EXACT_COVERS)]
    kind = [synth.LENS_COLUMN, synth.LENS_LINF, synth.LENS_PROJECTION, synth.LENS_L2][seed % 4]
    ax = synth.Axis(kind, nint, p, column=int(rng.integers(0, d)))
    if kind == synth.LENS_PROJECTION:
        ax.direction = (rng.integers(-4, 5, size=d) / 4.0).astype(np.float32)
    eps = [0.5, 0.75, 1.0, 1.25][seed % 4]
    params = synth.Params([ax], eps=eps, min_pts=int(rng.integers(1, 5)))
    # the L2 lens is a rounded square root, so its endpoints are exact only
    # when compared against the oracle's own FP64 cover
    _compare(X, params, exact_endpoints=(kind != synth.LENS_L2))


@pytest.mark.parametrize("seed", range(6))
def test_dyadic_2d_exact(seed):
    rng = np.random.default_rng(2000 + seed)
    n = int(rng.integers(8, 30))
    d = int(rng.integers(2, 4))
    X = synth.dyadic_cloud(rng, n, d)
    c1, c2 = EXACT_COVERS[seed % 6], EXACT_COVERS[(seed + 2) % 6]
    axes = [synth.Axis(synth.LENS_COLUMN, c1[0], c1[1], column=0),
            synth.Axis(synth.LENS_COLUMN, c2[0], c2[1], column=1)]
    params = synth.Params(axes, eps=0.75, min_pts=2)
    _compare(X, params)


@pytest.mark.parametrize("seed", range(6))
def test_general_cover_exact_decisions(seed):
    """Non-dyadic overlap: endpoints are the oracle's FP64 ones; membership,
    DBSCAN and the graph must still be exactly right for those endpoints."""
    rng = np.random.default_rng(3000 + seed)
    X = synth.dyadic_cloud(rng, 30, 3)
    ax = synth.Axis(synth.LENS_PROJECTION, int(rng.integers(2, 8)), float(rng.uniform(0.05, 0.7)))
    ax.direction = (rng.integers(-4, 5, size=3) / 4.0).astype(np.float32)
    params = synth.Params([ax], eps=1.0, min_pts=3)
    _compare(X, params, exact_endpoints=False)


def test_ties_are_inclusive():
    """Points at squared distance exactly eps^2 are neighbours and lens values
    exactly on an endpoint belong to both intervals (closed readings)."""
    X = np.array([[0.0, 0.0], [0.5, 0.0], [1.0, 0.0], [1.5, 0.0], [2.0, 0.0]], np.float32)
    # lens = x; 3 intervals, 50% overlap over [0, 2]: [0,1], [0.5,1.5], [1,2]
    params = synth.Params([synth.Axis(synth.LENS_COLUMN, 3, 0.5, column=0)], eps=0.5, min_pts=2)
    g, _ = _compare(X, params)
    assert g.lo[0].tolist() == [0.0, 0.5, 1.0]
    assert g.hi[0].tolist() == [1.0, 1.5, 2.0]
    sets = [sorted(s) for s in g.node_sets()]
    assert sets == [[0, 1, 2], [1, 2, 3], [2, 3, 4]]
    assert {(int(a), int(b)): int(w) for (a, b), w in zip(g.edges, g.edge_weights)} == \
        {(0, 1): 2, (0, 2): 1, (1, 2): 2}


def test_lens_error_bounds_random():
    """On non-dyadic data the FP64 lens is within the standard error bound
    gamma_d * sum|x_j v_j| of the exact value (sqrt adds half an ulp)."""
    rng = np.random.default_rng(7)
    X = (rng.standard_normal((40, 33)) * 10).astype(np.float32)
    v = synth.unit_vector(rng, 33)
    u = 2.0 ** -53
    gam = 33 * u / (1 - 33 * u)
    fp = O.lens(X, synth.Axis(synth.LENS_PROJECTION, 1, 0.0, direction=v))
    fl2 = O.lens(X, synth.Axis(synth.LENS_L2, 1, 0.0))
    fc = O.lens(X, synth.Axis(synth.LENS_COLUMN, 1, 0.0, column=5))
    fi = O.lens(X, synth.Axis(synth.LENS_LINF, 1, 0.0))
    for i in range(40):
        x = [F(float(a)) for a in X[i]]
        exact = sum(a * F(float(b)) for a, b in zip(x, v))
        bound = gam * float(sum(abs(a * F(float(b))) for a, b in zip(x, v)))
        assert abs(float(F(fp[i]) - exact)) <= bound
        S = sum(a * a for a in x)
        # |fl(S) - S| <= gam*S, then sqrt: relative error <= gam/2 + u (+ tiny)
        rel = abs(fl2[i] - float(S) ** 0.5) / float(S) ** 0.5
        assert rel <= gam / 2 + 2 * u
        assert fc[i] == float(X[i, 5])
        assert fi[i] == float(np.max(np.abs(X[i].astype(np.float64))))


def test_pair_distance_error_bound():
    """The canonical FP64 squared distance is within gamma_{2d} * D of the
    exact squared distance of the two float vectors."""
    rng = np.random.default_rng(8)
    u = 2.0 ** -53
    for d in (1, 2, 7, 64, 256):
        gam = 2 * d * u / (1 - 2 * d * u)
        for _ in range(10):
            x = (rng.standard_normal(d) * rng.uniform(0.1, 100)).astype(np.float32)
            y = (x + rng.standard_normal(d).astype(np.float32)).astype(np.float32)
            got = O.pair_d2(x, y)
            exact = sum((F(float(a)) - F(float(b))) ** 2 for a, b in zip(x, y))
            assert abs(F(got) - exact) <= F(gam) * exact


def test_cover_closed_forms():
    lo, hi = O.cover(0.0, 10.0, 4, 0.5)          # L = 10/2.5 = 4, step 2
    assert lo.tolist() == [0.0, 2.0, 4.0, 6.0] and hi.tolist() == [4.0, 6.0, 8.0, 10.0]
    lo, hi = O.cover(-3.0, 5.0, 1, 0.3)
    assert lo.tolist() == [-3.0] and hi.tolist() == [5.0]
    lo, hi = O.cover(1.0, 9.0, 4, 0.0)           # a partition into 4 equal pieces
    assert lo.tolist() == [1.0, 3.0, 5.0, 7.0] and hi.tolist() == [3.0, 5.0, 7.0, 9.0]
    lo, hi = O.cover(2.5, 2.5, 3, 0.4)           # degenerate range
    assert lo.tolist() == [2.5] * 3 and hi.tolist() == [2.5] * 3
    # general: equal lengths, overlap fraction p, exact ends
    rng = np.random.default_rng(9)
    for _ in range(50):
        m = float(rng.normal() * 10)
        M = m + float(rng.uniform(0.01, 100))
        n = int(rng.integers(2, 60))
        p = float(rng.uniform(0, 0.9))
        lo, hi = O.cover(m, M, n, p)
        L = (M - m) / (n - (n - 1) * p)
        assert lo[0] == m and hi[-1] == M
        assert np.allclose(hi - lo, L, rtol=1e-9, atol=1e-12 * abs(M))
        assert np.allclose((hi[:-1] - lo[1:]) / L, p, atol=1e-9)
        assert np.all(np.diff(lo) >= 0)


@pytest.mark.parametrize("bad", ["nint0", "ov1", "ovneg", "epsneg", "epsnan", "minpts0", "nan", "inf", "col",
                                 "range_overflow"])
def test_invalid_params(bad):
    X = np.zeros((10, 3), np.float32)
    X[:, 0] = np.arange(10)
    ax = synth.Axis(synth.LENS_COLUMN, 3, 0.2, column=0)
    eps, mp = 1.0, 2
    if bad == "nint0":
        ax.n_intervals = 0
    elif bad == "ov1":
        ax.overlap = 1.0
    elif bad == "ovneg":
        ax.overlap = -0.1
    elif bad == "epsneg":
        eps = -1.0
    elif bad == "epsnan":
        eps = float("nan")
    elif bad == "minpts0":
        mp = 0
    elif bad == "nan":
        X[3, 1] = np.nan
    elif bad == "inf":
        X[4, 2] = np.inf
    elif bad == "col":
        ax.column = 3
    elif bad == "range_overflow":           # M - m overflows FP64: no finite endpoints
        vals = np.zeros(10)
        vals[0], vals[1] = -1.5e308, 1.5e308
        ax = synth.Axis(synth.LENS_VALUES, 3, 0.2, values=vals)
    with pytest.raises(O.OracleError):
        O.mapper(X, synth.Params([ax], eps=eps, min_pts=mp))


@pytest.mark.parametrize("b_first", [False, True])
def test_border_goes_to_lowest_cluster(b_first):
    """A non-core point adjacent to core points of two clusters joins the one
    with the lower canonical id (the one whose smallest core index is lower)."""
    A = [0.0, 0.125, 0.25, 0.375, 0.5]
    B = [1.5, 1.625, 1.75, 1.875, 2.0]
    xs = (B + [1.0] + A) if b_first else (A + [1.0] + B)
    X = np.array([[x, 0.0] for x in xs], np.float32)
    params = synth.Params([synth.Axis(synth.LENS_COLUMN, 1, 0.0, column=1)], eps=0.5, min_pts=4)
    g, _ = _compare(X, params)
    border = 5
    assert not g.slot_core[border]
    first = set(range(5))            # whichever cluster comes first in index order
    sets = g.node_sets()
    assert sets[0] == first | {border} and border not in sets[1]


def test_all_pairs_distances():
    """orc_all_d2 (the checker of the GPU tile distances and of band
    soundness) gives the canonical squared distance of every ordered pair of
    the listed rows: exact on dyadic-grid points, where every FP64 step is
    exact; bit-equal to the one-pair chain (a separate loop over the original
    rows) on general data, within gamma_2d of the exact value; symmetric with
    a zero diagonal; rows in any order, repeats allowed."""
    rng = np.random.default_rng(11)
    Xd = synth.dyadic_cloud(rng, 30, 5)
    rows = rng.permutation(30)[:20].astype(np.int32)
    rows[7] = rows[3]                                      # a repeated row
    D = O.all_d2(Xd, rows)
    assert D.shape == (20, 20)
    for a in range(20):
        for b in range(20):
            x, y = Xd[rows[a]], Xd[rows[b]]
            assert F(D[a, b]) == sum((F(float(p)) - F(float(q))) ** 2 for p, q in zip(x, y))
    u = 2.0 ** -53
    for d in (1, 3, 64, 257):
        X = (rng.standard_normal((25, d)) * rng.uniform(0.5, 50)).astype(np.float32)
        r = rng.integers(0, 25, size=17).astype(np.int32)
        D = O.all_d2(X, r)
        assert np.array_equal(D, D.T)
        assert np.all(np.diag(D) == 0.0)
        gam = 2 * d * u / (1 - 2 * d * u)
        for a in range(17):
            for b in range(17):
                assert D[a, b] == O.pair_d2(X[r[a]], X[r[b]])
        for a, b in ((0, 1), (5, 16), (16, 2)):
            exact = sum((F(float(p)) - F(float(q))) ** 2 for p, q in zip(X[r[a]], X[r[b]]))
            assert abs(F(D[a, b]) - exact) <= F(gam) * exact
