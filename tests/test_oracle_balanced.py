"""Pins of the oracle's balanced cover (CPU): a worked example, the special
case where lens values equal their ranks (then it is the uniform cover of
[0, N-1] rounded outward), and invariants on random lens values with ties:
endpoints are lens values, monotone, cover every point, and every interval
holds between floor(L) + 1 and ceil(L) + 2 points of distinct values, where
L = (N - 1) / (n - (n - 1) p) is the rank length."""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03209_amd import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_worked_example():
    g = json.load(open(os.path.join(GOLDEN, "balanced_cover.json")))
    f = np.array(g["values"], np.float64)
    lo, hi = O.cover_balanced(f, g["n_intervals"], g["overlap"])
    assert lo.tolist() == g["lo"] and hi.tolist() == g["hi"]
    counts = [int(((f >= a) & (f <= b)).sum()) for a, b in zip(lo, hi)]
    assert counts == g["counts"]


@pytest.mark.parametrize("N,n,p", [(10, 3, 0.25), (1000, 7, 0.3), (37, 10, 0.5), (5, 8, 0.1), (2, 1, 0.0),
                                   (101, 20, 0.0), (64, 4, 0.75)])
def test_values_equal_ranks(N, n, p):
    """Lens values 0..N-1 in a random order: each endpoint is the rank itself,
    so the balanced cover is the uniform cover of [0, N-1] (the pinned
    closed form) rounded outward to integers."""
    f = np.random.default_rng(N + n).permutation(N).astype(np.float64)
    lo, hi = O.cover_balanced(f, n, p)
    ulo, uhi = O.cover(0.0, float(N - 1), n, p)
    assert lo.tolist() == [float(max(0, math.floor(x))) for x in ulo]
    assert hi.tolist() == [float(min(N - 1, math.ceil(x))) for x in uhi]


@pytest.mark.parametrize("seed", range(6))
def test_invariants(seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 3000))
    n = int(rng.integers(1, 40))
    p = float(rng.choice([0.0, 0.1, 0.3, 0.5, 0.9]))
    distinct = seed % 2 == 0
    f = rng.normal(size=N) if distinct else np.round(rng.normal(size=N), 1)   # odd seeds: many ties
    lo, hi = O.cover_balanced(f, n, p)
    vals = set(f.tolist())
    assert all(x in vals for x in lo) and all(x in vals for x in hi)
    assert np.all(np.diff(lo) >= 0) and np.all(np.diff(hi) >= 0) and np.all(lo <= hi)
    assert lo[0] == f.min() and hi[-1] == f.max()
    inside = np.zeros(N, bool)
    for a, b in zip(lo, hi):
        inside |= (f >= a) & (f <= b)
    assert inside.all()
    if distinct:
        L = (N - 1) / (n - (n - 1) * p)
        for a, b in zip(lo, hi):
            c = int(((f >= a) & (f <= b)).sum())
            assert math.floor(L) + 1 <= c <= math.ceil(L) + 2, (c, L)


def test_mapper_elements_follow_the_cover():
    """End to end: with cover = balanced the oracle's elements are the
    pullbacks of the balanced intervals (sizes equal the interval counts)."""
    w = synth.mixture_100k_d64(scale=0.02)
    w.params.axes[0].cover = 1
    g = O.mapper(w.X, w.params)
    f = g.lens[0]
    lo, hi = O.cover_balanced(f, w.params.axes[0].n_intervals, w.params.axes[0].overlap)
    assert np.array_equal(g.lo[0], lo) and np.array_equal(g.hi[0], hi)
    sizes = np.diff(g.elem_offsets)
    assert sizes.tolist() == [int(((f >= a) & (f <= b)).sum()) for a, b in zip(lo, hi)]
    assert sizes.max() - sizes.min() <= 3
