"""Exact rational mapper, written straight from the definitions, for tiny inputs.

Used only to pin the FP64 oracle.  Every quantity is a fractions.Fraction, so
there is no rounding anywhere except where a definition itself asks for a
double (the correctly rounded square root of the L2 lens), which is found by an
exact midpoint test rather than by calling a square-root routine.

Definitions followed (Background section of the paper): cover of the lens
image by n intervals of one length with fraction-p overlap; DBSCAN of each
pullback set (eps-ball closed, self counted, minPts); mapper graph = nerve of
the clusters (edge iff two clusters share a point).
"""
from __future__ import annotations

import math
from fractions import Fraction as F
from typing import List

import numpy as np

LENS_COLUMN, LENS_L2, LENS_LINF, LENS_PROJECTION, LENS_VALUES = 0, 1, 2, 3, 4


def correctly_rounded_sqrt(S: F) -> float:
    """The double nearest to sqrt(S), found by exact comparisons of squares
    against the rounding midpoints around a candidate."""
    if S == 0:
        return 0.0
    r = math.sqrt(float(S))
    for _ in range(4):
        up = math.nextafter(r, math.inf)
        dn = math.nextafter(r, 0.0)
        mid_hi = (F(r) + F(up)) / 2
        mid_lo = (F(r) + F(dn)) / 2
        if mid_hi * mid_hi < S:
            r = up
        elif mid_lo * mid_lo > S:
            r = dn
        else:
            return r
    raise AssertionError("no convergence")


def exact_lens(X: np.ndarray, axis) -> List:
    n, d = X.shape
    out = []
    for i in range(n):
        x = [F(float(v)) for v in X[i]]
        if axis.kind == LENS_COLUMN:
            out.append(x[axis.column])
        elif axis.kind == LENS_LINF:
            out.append(max(abs(v) for v in x))
        elif axis.kind == LENS_L2:
            out.append(F(correctly_rounded_sqrt(sum(v * v for v in x))))
        elif axis.kind == LENS_PROJECTION:
            out.append(sum(v * F(float(w)) for v, w in zip(x, axis.direction)))
        elif axis.kind == LENS_VALUES:
            out.append(F(float(axis.values[i])))
        else:
            raise ValueError(axis.kind)
    return out


def exact_cover(m: F, M: F, n: int, p: F):
    """n closed intervals of equal length L covering [m, M], consecutive ones
    sharing the fraction p of L: m + (n-1)(1-p)L + L = M."""
    L = (M - m) / (n - (n - 1) * p)
    s = L * (1 - p)
    lo = [m + k * s for k in range(n)]
    hi = [lo[k] + L for k in range(n)]
    return lo, hi


def exact_dbscan(P: List[List[F]], E: F, min_pts: int):
    """DBSCAN by definition: neighbours are points at squared distance <= E
    (the point itself included); core points have >= min_pts neighbours;
    clusters are connected components of core points; a non-core point with a
    core neighbour joins the lowest-numbered such cluster; cluster numbers
    follow the smallest core index of each component."""
    n = len(P)
    nb = [[sum((a - b) ** 2 for a, b in zip(P[i], P[j])) <= E for j in range(n)]
          for i in range(n)]
    count = [sum(row) for row in nb]
    core = [c >= min_pts for c in count]
    comp = [-1] * n
    ncomp = 0
    for s in range(n):                       # BFS from cores in index order
        if not core[s] or comp[s] >= 0:
            continue
        comp[s] = ncomp
        stack = [s]
        while stack:
            u = stack.pop()
            for v in range(n):
                if core[v] and nb[u][v] and comp[v] < 0:
                    comp[v] = ncomp
                    stack.append(v)
        ncomp += 1
    label = list(comp)
    for i in range(n):
        if not core[i]:
            cands = [comp[j] for j in range(n) if core[j] and nb[i][j]]
            label[i] = min(cands) if cands else -1
    return count, core, label


def exact_mapper(X: np.ndarray, params, endpoints=None):
    """Whole graph.  `endpoints` optionally supplies per-axis (lo, hi) as
    Fractions; by default they come from exact_cover."""
    n = X.shape[0]
    lens = [exact_lens(X, ax) for ax in params.axes]
    los, his = [], []
    for a, ax in enumerate(params.axes):
        if endpoints is not None:
            lo, hi = endpoints[a]
        else:
            lo, hi = exact_cover(min(lens[a]), max(lens[a]), ax.n_intervals, F(ax.overlap))
        los.append(lo)
        his.append(hi)
    shape = [ax.n_intervals for ax in params.axes]
    elements = []
    if len(shape) == 1:
        for k in range(shape[0]):
            elements.append([i for i in range(n) if los[0][k] <= lens[0][i] <= his[0][k]])
    else:
        for k1 in range(shape[0]):
            for k2 in range(shape[1]):
                elements.append([i for i in range(n)
                                 if los[0][k1] <= lens[0][i] <= his[0][k1]
                                 and los[1][k2] <= lens[1][i] <= his[1][k2]])
    E = F(float(params.eps)) ** 2
    Xf = [[F(float(v)) for v in row] for row in X]
    nodes, node_elem, slot_count, slot_core = [], [], [], []
    for e, mem in enumerate(elements):
        cnt, core, lab = exact_dbscan([Xf[i] for i in mem], E, params.min_pts)
        slot_count += cnt
        slot_core += core
        nc = 1 + max([l for l in lab] + [-1])
        for c in range(nc):
            nodes.append(sorted(mem[t] for t in range(len(mem)) if lab[t] == c))
            node_elem.append(e)
    edges = {}
    for a in range(len(nodes)):
        for b in range(a + 1, len(nodes)):
            w = len(set(nodes[a]) & set(nodes[b]))
            if w:
                edges[(a, b)] = w
    return dict(lens=lens, lo=los, hi=his, elements=elements, nodes=nodes,
                node_elem=node_elem, edges=edges, slot_count=slot_count,
                slot_core=slot_core)
