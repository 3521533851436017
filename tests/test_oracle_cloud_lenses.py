"""Pins of the oracle's whole-cloud lenses (CPU): the L-infinity eccentricity
(largest distance to another point) and the k-NN distance lens.

- eccentricity: exact rational brute force on dyadic clouds; it equals the
  pinned k-NN distance at k = n - 1; points on a line reach their farthest
  end (closed form);
- in the mapper, both lenses are the square roots of those squared
  distances, bit for bit, and the pullback sets follow them.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03209_amd import synth


@pytest.mark.parametrize("seed", range(4))
def test_eccentricity_bruteforce(seed):
    rng = np.random.default_rng(200 + seed)
    n, d = int(rng.integers(2, 30)), int(rng.integers(1, 5))
    X = (rng.integers(-16, 17, size=(n, d)) / 4.0).astype(np.float32)
    F = [[Fraction(float(v)) for v in row] for row in X]
    got = O.ecc_d2(X)
    for i in range(n):
        ref = max(sum((a - b) ** 2 for a, b in zip(F[i], F[j])) for j in range(n) if j != i)
        assert got[i] == float(ref)


def test_eccentricity_is_last_neighbour():
    X = np.random.default_rng(5).normal(size=(60, 7)).astype(np.float32)
    assert np.array_equal(O.ecc_d2(X), O.knn_d2(X, 59))


def test_eccentricity_on_a_line():
    t = np.random.default_rng(6).permutation(np.arange(-40, 41)).astype(np.float32) / 8.0
    X = np.stack([t, 2 * t, np.zeros_like(t)], axis=1)            # collinear, exact in binary
    far = np.maximum(np.abs(t - t.min()), np.abs(t - t.max())).astype(np.float64)
    assert np.array_equal(O.ecc_d2(X), 5.0 * far * far)


@pytest.mark.parametrize("kind,k", [(synth.LENS_ECCENTRICITY, 0), (synth.LENS_KNN_DISTANCE, 5)])
def test_mapper_lens(kind, k):
    w = synth.mixture_100k_d64(scale=0.01)
    X = np.ascontiguousarray(w.X[:, :16])
    params = synth.Params([synth.Axis(kind, 6, 0.3, column=k)], eps=6.0, min_pts=4)
    g = O.mapper(X, params)
    ref = np.sqrt(O.ecc_d2(X) if kind == synth.LENS_ECCENTRICITY else O.knn_d2(X, k))
    assert np.array_equal(g.lens[0], ref)
    f = g.lens[0]
    for e, (a, b) in enumerate(zip(g.lo[0], g.hi[0])):
        members = g.elem_members[g.elem_offsets[e]:g.elem_offsets[e + 1]]
        assert np.array_equal(np.sort(members), np.flatnonzero((f >= a) & (f <= b)))
