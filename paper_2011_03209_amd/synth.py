"""Seeded synthetic point clouds shaped like the paper's mapper workloads.

This module holds input generation only: it draws points, lens directions and
parameter sets, and contains none of the mapper arithmetic (no lens, cover,
distance or clustering code).  Both the GPU path's tests and the CPU oracle's
tests read their inputs from here.

The paper times its command-line mapper on activation vectors (ImageNet 512-D,
Cifar 256-D) and on i.i.d. uniform 128-D vectors (Scalability, "Datasets").
Those datasets are not available, so Gaussian mixtures of the same sizes and
dimensions stand in for them; the noisy circle stands in for the snowman-style
worked example of the Background section (a curve sampled with noise, a height
lens, a handful of intervals with 30% overlap).

Draw order for every mixture (fixed so that a config is reproducible from its
seed alone): means (K x d) -> labels (n) -> unit noise (n x d) -> background
points -> lens directions.  Random unit vectors are drawn as g ~ N(0, I_d),
normalised in float64, then stored as float32; the float32 vector *is* the lens
direction (it need not be exactly unit length).
"""
from __future__ import annotations

import dataclasses
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 2011032090

LENS_COLUMN = 0
LENS_L2 = 1
LENS_LINF = 2
LENS_PROJECTION = 3
LENS_VALUES = 4
LENS_KNN_DISTANCE = 5      # sqrt of the k-th nearest-neighbour squared distance (k = column)
LENS_ECCENTRICITY = 6      # sqrt of the largest squared distance to another point

PREC_FP32 = 0
PREC_BF16 = 1
PREC_BF16X3 = 2
PREC_FP16 = 3
PREC_FP16X3 = 4
PREC_AUTO = 5


@dataclasses.dataclass
class Axis:
    """One lens axis and its interval cover."""
    kind: int
    n_intervals: int
    overlap: float
    column: int = 0
    direction: Optional[np.ndarray] = None   # float32 (d,)
    values: Optional[np.ndarray] = None      # float64 (n,)
    cover: int = 0                           # 0: uniform intervals; 1: balanced (equal point counts)


@dataclasses.dataclass
class Params:
    axes: List[Axis]
    eps: float
    min_pts: int
    precision: int = PREC_FP32


@dataclasses.dataclass
class Workload:
    name: str
    X: np.ndarray            # float32 (n, d), C-contiguous
    params: Params
    labels: Optional[np.ndarray] = None   # mixture component of each point (-1: background)


def unit_vector(rng: np.random.Generator, d: int) -> np.ndarray:
    g = rng.standard_normal(d)            # float64
    g = g / np.sqrt(np.dot(g, g))
    return g.astype(np.float32)


def gaussian_mixture(rng: np.random.Generator, n: int, d: int, k: int,
                     mean_sd: float = 4.0, sigma: float = 1.0,
                     background_frac: float = 0.0):
    """Mixture of k isotropic Gaussians, means ~ N(0, mean_sd^2 I), equal weights
    (labels i.i.d. uniform), plus an optional uniform background in the
    per-coordinate bounding box of the Gaussian samples."""
    means = rng.normal(0.0, mean_sd, size=(k, d)).astype(np.float32)
    labels = rng.integers(0, k, size=n)
    X = rng.standard_normal((n, d), dtype=np.float32)
    if sigma != 1.0:
        X *= np.float32(sigma)
    X += means[labels]
    labels = labels.astype(np.int32)
    if background_frac > 0.0:
        nb = int(round(background_frac * n))
        lo = X.min(axis=0)
        hi = X.max(axis=0)
        B = rng.uniform(0.0, 1.0, size=(nb, d)).astype(np.float32)
        B = lo + B * (hi - lo)
        X = np.concatenate([X, B.astype(np.float32)], axis=0)
        labels = np.concatenate([labels, np.full(nb, -1, np.int32)])
    return np.ascontiguousarray(X, dtype=np.float32), labels


def noisy_circle(rng: np.random.Generator, n: int, sigma: float) -> np.ndarray:
    theta = rng.uniform(0.0, 2.0 * np.pi, size=n)
    P = np.stack([np.cos(theta), np.sin(theta)], axis=1)
    P = P + rng.normal(0.0, sigma, size=(n, 2))
    return np.ascontiguousarray(P, dtype=np.float32)


# ---------------------------------------------------------------------------
# The five workloads.  `scale` shrinks n (and nothing else) for fast tests.
# ---------------------------------------------------------------------------

def circle_2k(scale: float = 1.0) -> Workload:
    """2,000 points on the unit circle + N(0, 0.02^2 I); y lens; 10 intervals,
    30% overlap; eps 0.1, minPts 5."""
    rng = np.random.default_rng(SEED_BASE + 1)
    n = max(8, int(round(2000 * scale)))
    X = noisy_circle(rng, n, 0.02)
    p = Params([Axis(LENS_COLUMN, 10, 0.3, column=1)], eps=0.1, min_pts=5)
    return Workload("circle2k_d2", X, p)


def mixture_100k_d64(scale: float = 1.0) -> Workload:
    """100,000 points in R^64, 20 Gaussians; L2 lens; 20 intervals, 25% overlap;
    eps 12.5, minPts 10."""
    rng = np.random.default_rng(SEED_BASE + 2)
    n = max(16, int(round(100_000 * scale)))
    X, lab = gaussian_mixture(rng, n, 64, 20)
    p = Params([Axis(LENS_L2, 20, 0.25)], eps=12.5, min_pts=10)
    return Workload("mix100k_d64", X, p, lab)


def mixture_1m_d256(scale: float = 1.0, precision: int = PREC_BF16X3) -> Workload:
    """1,000,000 points in R^256, 50 Gaussians; projection on a seeded unit
    vector; 40 intervals, 30% overlap; eps 24, minPts 10."""
    rng = np.random.default_rng(SEED_BASE + 3)
    n = max(16, int(round(1_000_000 * scale)))
    X, lab = gaussian_mixture(rng, n, 256, 50)
    v = unit_vector(rng, 256)
    p = Params([Axis(LENS_PROJECTION, 40, 0.3, direction=v)], eps=24.0, min_pts=10,
               precision=precision)
    return Workload("mix1m_d256", X, p, lab)


def mixture_500k_d128_2d(scale: float = 1.0, precision: int = PREC_FP16X3) -> Workload:
    """500,000 points in R^128, 30 Gaussians + 5% uniform background; 2-D lens of
    two seeded projections; 15x15 grid, 50% overlap; eps 17, minPts 8."""
    rng = np.random.default_rng(SEED_BASE + 4)
    n = max(16, int(round(500_000 * scale)))
    X, lab = gaussian_mixture(rng, n, 128, 30, background_frac=0.05)
    v1 = unit_vector(rng, 128)
    v2 = unit_vector(rng, 128)
    p = Params([Axis(LENS_PROJECTION, 15, 0.5, direction=v1),
                Axis(LENS_PROJECTION, 15, 0.5, direction=v2)], eps=17.0, min_pts=8,
               precision=precision)
    return Workload("mix500k_d128_grid", X, p, lab)


SERVING_CLOUDS = [(10_000, 32), (10_000, 256), (50_000, 64), (50_000, 128),
                  (200_000, 32), (200_000, 256), (500_000, 64), (500_000, 128)]


def serving_clouds(scale: float = 1.0, k: int = 20) -> List[np.ndarray]:
    """Eight resident Gaussian-mixture clouds (each n twice, each d twice)."""
    rng = np.random.default_rng(SEED_BASE + 5)
    out = []
    for n, d in SERVING_CLOUDS:
        m = max(16, int(round(n * scale)))
        X, _ = gaussian_mixture(rng, m, d, k)
        out.append(X)
    return out


def serving_requests(clouds: Sequence[np.ndarray], count: int, qps: float,
                     precision: int = PREC_BF16X3, seed: int = SEED_BASE + 50):
    """Poisson arrival times and random parameter sets over the given clouds.

    Each request: lens in {L2, random projection}, intervals U{5..50}, overlap
    U[0.1, 0.5], eps = 1.05*sqrt(2d), minPts U{5..20}."""
    rng = np.random.default_rng(seed)
    t = 0.0
    reqs = []
    for _ in range(count):
        t += rng.exponential(1.0 / qps) if qps > 0 else 0.0
        c = int(rng.integers(0, len(clouds)))
        d = clouds[c].shape[1]
        kind = LENS_L2 if rng.integers(0, 2) == 0 else LENS_PROJECTION
        nint = int(rng.integers(5, 51))
        ov = float(rng.uniform(0.1, 0.5))
        eps = 1.05 * float(np.sqrt(2.0 * d))
        mp = int(rng.integers(5, 21))
        direction = unit_vector(rng, d) if kind == LENS_PROJECTION else None
        p = Params([Axis(kind, nint, ov, direction=direction)], eps=eps, min_pts=mp,
                   precision=precision)
        reqs.append((t, c, p))
    return reqs


def dyadic_cloud(rng: np.random.Generator, n: int, d: int, grid: int = 8,
                 span: int = 16) -> np.ndarray:
    """Points whose coordinates are multiples of 1/grid with |x| <= span/grid.
    Every float64 sum of squares and products of such values is exact, so the
    oracle's arithmetic can be compared with exact rationals, ties included."""
    Z = rng.integers(-span, span + 1, size=(n, d))
    return np.ascontiguousarray(Z.astype(np.float32) / np.float32(grid))


def blobs(rng: np.random.Generator, n: int, d: int, k: int, sep: float,
          sigma: float = 1.0):
    """k well-separated Gaussian blobs: centres at sep * (distinct axes)."""
    centres = np.zeros((k, d), np.float64)
    for c in range(k):
        centres[c, c % d] = sep * (1 + c // d)
    lab = rng.integers(0, k, size=n)
    X = centres[lab] + rng.normal(0.0, sigma, size=(n, d))
    return np.ascontiguousarray(X, dtype=np.float32), lab.astype(np.int32)
