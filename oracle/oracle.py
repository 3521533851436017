"""Python view of the plain FP64 CPU mapper in mapper_oracle.c.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the product library.  It marshals numpy
arrays into the C oracle and copies its results back; it computes nothing
itself.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import List, Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mapper_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O3", "-ffp-contract=off", "-fno-fast-math", "-march=x86-64-v3",
          "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc.  Contraction stays off so each expression
    rounds exactly as written; -march=x86-64-v3 lets fma() be a single
    correctly rounded instruction."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.run(["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, LIB)
    return LIB


class _Axis(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("column", ctypes.c_int32),
                ("direction", ctypes.POINTER(ctypes.c_float)),
                ("values", ctypes.POINTER(ctypes.c_double)),
                ("n_intervals", ctypes.c_int32), ("overlap", ctypes.c_double),
                ("cover", ctypes.c_int32)]


class _Graph(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int64), ("n_edges", ctypes.c_int64),
                ("n_elements", ctypes.c_int64), ("n_slots", ctypes.c_int64),
                ("node_element", ctypes.POINTER(ctypes.c_int32)),
                ("node_offsets", ctypes.POINTER(ctypes.c_int64)),
                ("node_members", ctypes.POINTER(ctypes.c_int32)),
                ("edges", ctypes.POINTER(ctypes.c_int32)),
                ("edge_weights", ctypes.POINTER(ctypes.c_int32)),
                ("lens", ctypes.POINTER(ctypes.c_double)),
                ("lo", ctypes.POINTER(ctypes.c_double)),
                ("hi", ctypes.POINTER(ctypes.c_double)),
                ("elem_offsets", ctypes.POINTER(ctypes.c_int64)),
                ("elem_members", ctypes.POINTER(ctypes.c_int32)),
                ("slot_count", ctypes.POINTER(ctypes.c_int32)),
                ("slot_core", ctypes.POINTER(ctypes.c_uint8)),
                ("slot_node", ctypes.POINTER(ctypes.c_int32))]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.orc_mapper.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.POINTER(_Axis), ctypes.c_double,
                                 ctypes.c_int32, ctypes.POINTER(ctypes.POINTER(_Graph))]
        L.orc_mapper.restype = ctypes.c_int
        L.orc_graph_free.argtypes = [ctypes.POINTER(_Graph)]
        L.orc_graph_free.restype = None
        L.orc_lens.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int64, ctypes.c_int32,
                               ctypes.POINTER(_Axis), ctypes.POINTER(ctypes.c_double)]
        L.orc_lens.restype = ctypes.c_int
        L.orc_cover.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
        L.orc_cover.restype = None
        L.orc_cover_balanced.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.c_int64, ctypes.c_int32,
                                         ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_double)]
        L.orc_cover_balanced.restype = ctypes.c_int
        L.orc_dbscan.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, ctypes.c_double,
                                 ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                 ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_int32)]
        L.orc_dbscan.restype = ctypes.c_int64
        L.orc_knn_d2.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_double)]
        L.orc_knn_d2.restype = ctypes.c_int
        L.orc_knn_d2_rows.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int64, ctypes.c_int32,
                                      ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_double)]
        L.orc_knn_d2_rows.restype = ctypes.c_int
        L.orc_ecc_d2.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int64, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_double)]
        L.orc_ecc_d2.restype = ctypes.c_int
        L.orc_pair_d2.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                  ctypes.c_int32]
        L.orc_pair_d2.restype = ctypes.c_double
        L.orc_all_d2.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_int64, ctypes.c_int32,
                                 ctypes.POINTER(ctypes.c_int32), ctypes.c_int64, ctypes.POINTER(ctypes.c_double)]
        L.orc_all_d2.restype = ctypes.c_int
        L.orc_threads.argtypes = []
        L.orc_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle returned {code}")
        self.code = code


@dataclasses.dataclass
class Graph:
    """Mapper graph plus the per-stage intermediate values the oracle saw."""
    node_element: np.ndarray
    node_offsets: np.ndarray
    node_members: np.ndarray
    edges: np.ndarray          # (E, 2) int32, a < b, lexicographic
    edge_weights: np.ndarray
    lens: np.ndarray           # (n_axes, n) float64
    lo: List[np.ndarray]
    hi: List[np.ndarray]
    elem_offsets: np.ndarray
    elem_members: np.ndarray
    slot_count: np.ndarray
    slot_core: np.ndarray
    slot_node: np.ndarray

    @property
    def n_nodes(self) -> int:
        return int(self.node_element.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])

    def node_sets(self):
        o = self.node_offsets
        return [set(self.node_members[o[v]:o[v + 1]].tolist()) for v in range(self.n_nodes)]


def _axes(params, keep):
    arr = (_Axis * len(params.axes))()
    for a, ax in enumerate(params.axes):
        arr[a].kind = ax.kind
        arr[a].column = ax.column
        arr[a].n_intervals = ax.n_intervals
        arr[a].overlap = ax.overlap
        arr[a].cover = getattr(ax, "cover", 0)
        if ax.direction is not None:
            v = np.ascontiguousarray(ax.direction, dtype=np.float32)
            keep.append(v)
            arr[a].direction = _p(v, ctypes.c_float)
        if ax.values is not None:
            v = np.ascontiguousarray(ax.values, dtype=np.float64)
            keep.append(v)
            arr[a].values = _p(v, ctypes.c_double)
    return arr


def _copy(ptr, count, dtype):
    if count <= 0:
        return np.zeros(0, dtype)
    return np.ctypeslib.as_array(ptr, shape=(int(count),)).astype(dtype, copy=True)


def mapper(X: np.ndarray, params) -> Graph:
    """Whole mapper graph of X under params (a synth.Params)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    keep: list = []
    axes = _axes(params, keep)
    out = ctypes.POINTER(_Graph)()
    rc = lib().orc_mapper(_p(X, ctypes.c_float), n, d, len(params.axes), axes,
                          float(params.eps), int(params.min_pts), ctypes.byref(out))
    if rc != 0:
        raise OracleError(rc)
    g = out.contents
    try:
        nn, ne, nel, ns = g.n_nodes, g.n_edges, g.n_elements, g.n_slots
        node_off = _copy(g.node_offsets, nn + 1, np.int64)
        lens = _copy(g.lens, n * len(params.axes), np.float64).reshape(len(params.axes), n)
        lo_all = _copy(g.lo, sum(a.n_intervals for a in params.axes), np.float64)
        hi_all = _copy(g.hi, sum(a.n_intervals for a in params.axes), np.float64)
        lo, hi, o = [], [], 0
        for ax in params.axes:
            lo.append(lo_all[o:o + ax.n_intervals])
            hi.append(hi_all[o:o + ax.n_intervals])
            o += ax.n_intervals
        res = Graph(
            node_element=_copy(g.node_element, nn, np.int32),
            node_offsets=node_off,
            node_members=_copy(g.node_members, int(node_off[-1]), np.int32),
            edges=_copy(g.edges, 2 * ne, np.int32).reshape(ne, 2),
            edge_weights=_copy(g.edge_weights, ne, np.int32),
            lens=lens, lo=lo, hi=hi,
            elem_offsets=_copy(g.elem_offsets, nel + 1, np.int64),
            elem_members=_copy(g.elem_members, ns, np.int32),
            slot_count=_copy(g.slot_count, ns, np.int32),
            slot_core=_copy(g.slot_core, ns, np.uint8),
            slot_node=_copy(g.slot_node, ns, np.int32),
        )
    finally:
        lib().orc_graph_free(out)
    return res


def lens(X: np.ndarray, axis) -> np.ndarray:
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    keep: list = []

    class _P:
        axes = [axis]
    arr = _axes(_P, keep)
    f = np.zeros(n, np.float64)
    rc = lib().orc_lens(_p(X, ctypes.c_float), n, d, arr, _p(f, ctypes.c_double))
    if rc != 0:
        raise OracleError(rc)
    return f


def cover(m: float, M: float, n_intervals: int, overlap: float):
    lo = np.zeros(n_intervals, np.float64)
    hi = np.zeros(n_intervals, np.float64)
    lib().orc_cover(float(m), float(M), int(n_intervals), float(overlap),
                    _p(lo, ctypes.c_double), _p(hi, ctypes.c_double))
    return lo, hi


def cover_balanced(f: np.ndarray, n_intervals: int, overlap: float):
    """Balanced cover of the lens values f: intervals holding equal numbers
    of points (the uniform cover on the rank axis, rounded outward)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    lo = np.zeros(n_intervals, np.float64)
    hi = np.zeros(n_intervals, np.float64)
    rc = lib().orc_cover_balanced(_p(f, ctypes.c_double), f.size, int(n_intervals), float(overlap),
                                  _p(lo, ctypes.c_double), _p(hi, ctypes.c_double))
    if rc != 0:
        raise OracleError(rc)
    return lo, hi


def dbscan(X: np.ndarray, members: np.ndarray, eps: float, min_pts: int):
    """DBSCAN of the points X[members] (members ascending).  Returns
    (count, core, cluster id or -1)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    idx = np.ascontiguousarray(members, dtype=np.int32)
    nk = idx.shape[0]
    cnt = np.zeros(max(nk, 1), np.int32)
    core = np.zeros(max(nk, 1), np.uint8)
    cid = np.zeros(max(nk, 1), np.int32)
    rc = lib().orc_dbscan(_p(X, ctypes.c_float), X.shape[1], _p(idx, ctypes.c_int32), nk,
                          float(eps), int(min_pts), _p(cnt, ctypes.c_int32),
                          _p(core, ctypes.c_uint8), _p(cid, ctypes.c_int32))
    if rc < 0:
        raise OracleError(int(rc))
    return cnt[:nk], core[:nk].astype(bool), cid[:nk]


def knn_d2(X: np.ndarray, k: int) -> np.ndarray:
    """k-th smallest canonical squared distance from each point to the others."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    out = np.zeros(n, np.float64)
    rc = lib().orc_knn_d2(_p(X, ctypes.c_float), n, d, int(k), _p(out, ctypes.c_double))
    if rc != 0:
        raise OracleError(rc)
    return out


def knn_d2_rows(X: np.ndarray, k: int, rows) -> np.ndarray:
    """knn_d2 for the listed rows only."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    r = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.zeros(r.size, np.float64)
    rc = lib().orc_knn_d2_rows(_p(X, ctypes.c_float), n, d, int(k), _p(r, ctypes.c_int32), r.size,
                               _p(out, ctypes.c_double))
    if rc != 0:
        raise OracleError(rc)
    return out


def ecc_d2(X: np.ndarray) -> np.ndarray:
    """Largest canonical squared distance from each point to the others."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    n, d = X.shape
    out = np.zeros(n, np.float64)
    rc = lib().orc_ecc_d2(_p(X, ctypes.c_float), n, d, _p(out, ctypes.c_double))
    if rc != 0:
        raise OracleError(rc)
    return out


def pair_d2(x: np.ndarray, y: np.ndarray) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    return float(lib().orc_pair_d2(_p(x, ctypes.c_float), _p(y, ctypes.c_float), x.shape[0]))


def all_d2(X: np.ndarray, rows) -> np.ndarray:
    """Canonical squared distances of all ordered pairs of X[rows] (m x m)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    r = np.ascontiguousarray(rows, dtype=np.int32)
    out = np.empty((r.shape[0], r.shape[0]), np.float64)
    rc = lib().orc_all_d2(_p(X, ctypes.c_float), X.shape[0], X.shape[1], _p(r, ctypes.c_int32), r.shape[0],
                          _p(out, ctypes.c_double))
    if rc != 0:
        raise ValueError(f"orc_all_d2 failed ({rc})")
    return out


def threads() -> int:
    """OpenMP threads the oracle's parallel loops run on."""
    return int(lib().orc_threads())
