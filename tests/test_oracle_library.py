"""Pins of the FP64 oracle against libraries, closed forms and invariants (CPU).

- scikit-learn DBSCAN (brute force): same core points and the same partition
  of the core points (border points are not compared: scikit-learn assigns
  them in visiting order);
- scipy connected components: with minPts = 1 every point is core and the
  clusters are the connected components of the eps-graph;
- closed forms: the noisy circle gives a single 18-cycle; a huge eps gives the
  nerve of the interval cover; a single interval gives no edges;
- invariants: node lens values lie in their element's box, nodes of one element
  are disjoint, every member is core or eps-adjacent to a core of its node,
  edge iff shared point with weight = |intersection|, separated blobs never
  share a component.
"""
import json
import os

import networkx as nx
import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import connected_components
from sklearn.cluster import DBSCAN

from oracle import oracle as O
from paper_2011_03209_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _d2_numpy(P):
    """Independent FP64 squared distances (direct differences, numpy order)."""
    P = P.astype(np.float64)
    diff = P[:, None, :] - P[None, :, :]
    return np.einsum("ijk,ijk->ij", diff, diff)


def _far_from_ties(P, eps, rel=1e-9):
    D = _d2_numpy(P)
    E = eps * eps
    return not np.any(np.abs(D - E) <= rel * E)


def _partition(labels, mask):
    groups = {}
    for i in np.nonzero(mask)[0]:
        groups.setdefault(int(labels[i]), set()).add(int(i))
    return sorted(sorted(s) for s in groups.values())


@pytest.mark.parametrize("seed", range(8))
def test_core_partition_matches_sklearn(seed):
    rng = np.random.default_rng(100 + seed)
    d = int(rng.integers(2, 17))
    n = int(rng.integers(50, 400))
    X, _ = synth.gaussian_mixture(rng, n, d, int(rng.integers(2, 6)), mean_sd=3.0)
    eps = float(np.sqrt(2 * d) * rng.uniform(0.6, 1.2))
    if not _far_from_ties(X, eps):
        pytest.skip("pair too close to eps for a float library comparison")
    mp = int(rng.integers(2, 12))
    cnt, core, cid = O.dbscan(X, np.arange(n, dtype=np.int32), eps, mp)
    sk = DBSCAN(eps=eps, min_samples=mp, algorithm="brute").fit(X.astype(np.float64))
    sk_core = np.zeros(n, bool)
    sk_core[sk.core_sample_indices_] = True
    assert np.array_equal(core, sk_core)
    assert _partition(cid, core) == _partition(sk.labels_, sk_core)
    # every border point is adjacent to a core point of its cluster
    D = _d2_numpy(X)
    for i in np.nonzero(~core)[0]:
        if cid[i] >= 0:
            assert np.any(core & (cid == cid[i]) & (D[i] <= eps * eps))
        else:
            assert not np.any(core & (D[i] <= eps * eps))
    assert np.array_equal(cnt, (D <= eps * eps).sum(axis=1))


@pytest.mark.parametrize("seed", range(5))
def test_minpts1_is_connected_components(seed):
    rng = np.random.default_rng(200 + seed)
    d = int(rng.integers(1, 9))
    n = int(rng.integers(30, 300))
    X = (rng.uniform(0, 10, size=(n, d))).astype(np.float32)
    eps = float(rng.uniform(0.3, 2.0))
    if not _far_from_ties(X, eps):
        pytest.skip("pair too close to eps")
    cnt, core, cid = O.dbscan(X, np.arange(n, dtype=np.int32), eps, 1)
    assert core.all()
    A = csr_matrix(_d2_numpy(X) <= eps * eps)
    nc, lab = connected_components(A, directed=False)
    assert cid.max() + 1 == nc
    # canonical numbering: components ordered by their smallest member
    first = {}
    for i, l in enumerate(lab):
        first.setdefault(l, i)
    order = {l: r for r, l in enumerate(sorted(first, key=first.get))}
    assert np.array_equal(cid, np.array([order[l] for l in lab]))


def test_circle_closed_form():
    """A noisy circle with a height lens: one node in each end interval, two
    arcs in each of the 8 middle ones; consecutive arcs overlap, so the mapper
    graph is one cycle of 18 nodes."""
    with open(os.path.join(GOLDEN, "circle_cycle.json")) as fh:
        gold = json.load(fh)
    w = synth.circle_2k()
    g = O.mapper(w.X, w.params)
    G = nx.Graph()
    G.add_nodes_from(range(g.n_nodes))
    G.add_edges_from(g.edges.tolist())
    assert g.n_nodes == gold["nodes"]
    assert g.n_edges == gold["edges"]
    assert nx.number_connected_components(G) == gold["components"]
    assert set(dict(G.degree()).values()) == {2}
    assert len(nx.cycle_basis(G)) == gold["cycle_rank"]
    # one node per end interval, two per middle interval
    per_elem = np.bincount(g.node_element, minlength=10)
    assert per_elem.tolist() == [1] + [2] * 8 + [1]


def test_huge_eps_gives_nerve_of_cover():
    """eps above the diameter and minPts = 1: each nonempty element is one
    cluster, so the graph is the nerve of the pullback sets; with p < 1/2 only
    consecutive intervals can share points."""
    rng = np.random.default_rng(5)
    X = rng.normal(size=(500, 5)).astype(np.float32)
    ax = synth.Axis(synth.LENS_COLUMN, 12, 0.3, column=2)
    g = O.mapper(X, synth.Params([ax], eps=1e3, min_pts=1))
    f = X[:, 2].astype(np.float64)
    lo, hi = g.lo[0], g.hi[0]
    inside = [(lo[k] <= f) & (f <= hi[k]) for k in range(12)]
    nonempty = [k for k in range(12) if inside[k].any()]
    assert g.node_element.tolist() == nonempty
    node_of = {k: v for v, k in enumerate(nonempty)}
    want = {}
    for k in range(11):
        w = int((inside[k] & inside[k + 1]).sum())
        if w:
            want[(node_of[k], node_of[k + 1])] = w
    got = {(int(a), int(b)): int(c) for (a, b), c in zip(g.edges, g.edge_weights)}
    assert got == want


def test_single_interval_no_edges():
    rng = np.random.default_rng(6)
    X, _ = synth.gaussian_mixture(rng, 400, 4, 3, mean_sd=6.0)
    eps = 1.6
    if not _far_from_ties(X, eps):
        pytest.skip("tie")
    g = O.mapper(X, synth.Params([synth.Axis(synth.LENS_L2, 1, 0.0)], eps=eps, min_pts=5))
    assert g.n_edges == 0
    sk = DBSCAN(eps=eps, min_samples=5, algorithm="brute").fit(X.astype(np.float64))
    core = np.zeros(400, bool)
    core[sk.core_sample_indices_] = True
    got = sorted(sorted(s & set(np.nonzero(core)[0].tolist())) for s in g.node_sets())
    assert got == _partition(sk.labels_, core)


def test_degenerate_range_every_point_everywhere():
    X = np.zeros((20, 3), np.float32)
    X[:, 1] = np.linspace(0, 1, 20, dtype=np.float32)
    ax = synth.Axis(synth.LENS_COLUMN, 4, 0.25, column=0)    # lens constant 0
    g = O.mapper(X, synth.Params([ax], eps=0.2, min_pts=2))
    assert g.node_element.tolist() == [0, 1, 2, 3]
    assert all(s == set(range(20)) for s in g.node_sets())
    assert g.n_edges == 6 and set(g.edge_weights.tolist()) == {20}


def test_separated_blobs():
    rng = np.random.default_rng(11)
    X, lab = synth.blobs(rng, 1500, 8, 5, sep=50.0)
    ax = synth.Axis(synth.LENS_L2, 8, 0.3)
    g = O.mapper(X, synth.Params([ax], eps=4.5, min_pts=5))
    G = nx.Graph()
    G.add_nodes_from(range(g.n_nodes))
    G.add_edges_from(g.edges.tolist())
    sets = g.node_sets()
    for comp in nx.connected_components(G):
        pts = set().union(*(sets[v] for v in comp))
        assert len(set(lab[list(pts)].tolist())) == 1
    blobs_seen = {int(lab[next(iter(sets[v]))]) for v in range(g.n_nodes)}
    assert nx.number_connected_components(G) == len(blobs_seen) == 5


def test_structural_invariants_mixture():
    w = synth.mixture_100k_d64(scale=0.02)
    g = O.mapper(w.X, w.params)
    f = g.lens[0]
    lo, hi = g.lo[0], g.hi[0]
    E = w.params.eps ** 2
    sets = g.node_sets()
    no = g.node_offsets
    for v in range(g.n_nodes):
        e = int(g.node_element[v])
        mem = g.node_members[no[v]:no[v + 1]]
        assert np.all(np.diff(mem) > 0)
        assert np.all((lo[e] <= f[mem]) & (f[mem] <= hi[e]))
    for e in np.unique(g.node_element):
        vs = np.nonzero(g.node_element == e)[0]
        for i in range(len(vs)):
            for j in range(i + 1, len(vs)):
                assert not (sets[vs[i]] & sets[vs[j]])
    # each member is core or eps-adjacent (independent numpy FP64) to a core of its node
    eo = g.elem_offsets
    for e in range(len(eo) - 1):
        mem = g.elem_members[eo[e]:eo[e + 1]]
        if len(mem) == 0:
            continue
        D = _d2_numpy(w.X[mem])
        core = g.slot_core[eo[e]:eo[e + 1]].astype(bool)
        node = g.slot_node[eo[e]:eo[e + 1]]
        near = np.abs(D - E) <= 1e-9 * E
        for t in range(len(mem)):
            if node[t] < 0 or core[t]:
                continue
            ok = core & (node == node[t]) & ((D[t] <= E) | near[t])
            assert ok.any()
    want = {}
    for a in range(g.n_nodes):
        for b in range(a + 1, g.n_nodes):
            k = len(sets[a] & sets[b])
            if k:
                want[(a, b)] = k
    got = {(int(a), int(b)): int(c) for (a, b), c in zip(g.edges, g.edge_weights)}
    assert got == want
