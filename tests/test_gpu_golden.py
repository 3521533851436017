"""Whole mapper graphs at the paper-scale sizes against the oracle (needs an
MI355X).

The oracle's graphs of the two large workloads -- 1,000,000 x 256 (projection
lens, 40 intervals) and 525,000 x 128 (two projection lenses, 15 x 15 grid
cover) -- take the FP64 CPU oracle tens of CPU-minutes each, so
oracle/make_golden.py ran them once and stored SHA-256 digests of every
canonical array (nodes, members, edges, weights) and of every stage array
(lens, endpoints, pullback sets, neighbour counts, core flags, node labels),
with per-element digests (tests/golden/*.json).  Here the GPU graph of the
same seeded cloud is digested the same way in the launch configurations the
benchmark times and must match digest for digest: the mapper graph is the
nerve of the DBSCAN clusters of each pullback set (Background section), and
every precision must give exactly the oracle's.
"""
import json
import os

import numpy as np
import pytest

from oracle.make_golden import digest_graph, golden_path
from paper_2011_03209_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_03209_amd import binding
    c = binding.Context(arena_bytes=96 << 30)
    yield c
    c.close()


def gpu_arrays(g) -> dict:
    s = g.stages
    return {"node_element": g.node_element, "node_offsets": g.node_offsets, "node_members": g.node_members,
            "edges": g.edges, "edge_weights": g.edge_weights, "lens": s["lens"], "lo": s["lo"], "hi": s["hi"],
            "elem_offsets": s["elem_offsets"], "elem_members": s["elem_members"],
            "slot_count": s["slot_count"], "slot_core": s["slot_core"], "slot_node": s["slot_node"]}


def compare(dg, gold, what):
    assert dg["n_elements"] == gold["n_elements"], what
    bad = [e for e, (a, b) in enumerate(zip(dg["elements"], gold["elements"])) if a != b]
    assert not bad, f"{what}: {len(bad)} elements differ, first {bad[0]}: {dg['elements'][bad[0]]} vs " \
                    f"{gold['elements'][bad[0]]}"
    for k in ("n_nodes", "n_edges", "n_slots"):
        assert dg[k] == gold[k], (what, k, dg[k], gold[k])
    for k, v in gold["sha256"].items():
        assert dg["sha256"][k] == v, (what, k)


NO_SCREEN = 8    # MAPPER_FLAG_NO_SCREEN: every tile pair (single 16-bit products then run as macro tiles)

WORKLOADS = {
    "mix1m_d256": (synth.mixture_1m_d256,
                   [(synth.PREC_BF16X3, 0), (synth.PREC_FP16X3, 0), (synth.PREC_FP16, 0),
                    (synth.PREC_FP16, NO_SCREEN), (synth.PREC_BF16, 0), (synth.PREC_FP32, 0)]),
    "mix500k_d128_grid": (synth.mixture_500k_d128_2d,
                          [(synth.PREC_BF16X3, 0), (synth.PREC_FP16X3, 0), (synth.PREC_FP16, 0),
                           (synth.PREC_FP16, NO_SCREEN), (synth.PREC_FP32, 0)]),
}


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_full_size_graph_is_the_oracles(ctx, name):
    """Every canonical array of the whole graph and of every stage, in each
    precision, screened (the default, as the benchmark runs) and unscreened
    (every tile pair, as macro tiles), has the oracle's digest."""
    with open(golden_path(name)) as fh:
        gold = json.load(fh)
    make, runs = WORKLOADS[name]
    w = make()
    cloud = ctx.cloud(w.X)
    try:
        for prec, flags in runs:
            print(f"[case] {name} prec={prec} flags={flags}", flush=True)
            p = w.params
            p.precision = prec
            g = cloud.run(p, debug=True, flags=flags)
            compare(digest_graph(gpu_arrays(g)), gold, f"{name} prec={prec} flags={flags}")
    finally:
        cloud.destroy()
