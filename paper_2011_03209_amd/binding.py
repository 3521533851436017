"""Python binding of libmapper_gpu (include/mapper_gpu.h), argument marshalling only.

Every stage of the mapper runs inside the HIP library; this module only turns
numpy / torch arguments into the C structs, and PyTorch only provides the
device arena and the HIP stream(s).  There is no CPU fallback: if the built
library is missing the import fails.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Dict, List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmapper_gpu.so")

MAPPER_OK, MAPPER_EINVAL, MAPPER_ENOMEM, MAPPER_EDEVICE = 0, -1, -2, -3
MAPPER_EBUSY, MAPPER_ETIMEDOUT, MAPPER_ENOTIMPL = -4, -5, -6
FLAG_DEBUG_STAGES = 1
FLAG_TILE_PAIRS = 2         # force one workgroup per 128 x 128 tile pair
FLAG_TILE_MACRO = 4         # force macro tiles (single 16-bit products)
FLAG_NO_SCREEN = 8          # compute every tile pair (no screening by cells)
MAX_EPS_VALUES = 4          # MAPPER_MAX_EPS_VALUES
MAX_MINPTS_VALUES = 16      # MAPPER_MAX_MINPTS_VALUES

PREC_NAMES = {0: "fp32", 1: "bf16", 2: "bf16x3", 3: "fp16", 4: "fp16x3", 5: "auto"}


class MapperError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"mapper error {code}: {msg}")
        self.code = code


class _Axis(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("column", ctypes.c_int32),
                ("direction", ctypes.POINTER(ctypes.c_float)),
                ("values", ctypes.POINTER(ctypes.c_double)),
                ("n_intervals", ctypes.c_int32), ("overlap", ctypes.c_double),
                ("cover", ctypes.c_int32)]


class _Params(ctypes.Structure):
    _fields_ = [("n_axes", ctypes.c_int32), ("axis", _Axis * 2), ("eps", ctypes.c_double),
                ("min_pts", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("flags", ctypes.c_uint32)]


class RunStats(ctypes.Structure):
    _fields_ = [("ms_total", ctypes.c_double), ("ms_lens", ctypes.c_double),
                ("ms_bin", ctypes.c_double), ("ms_tiles", ctypes.c_double),
                ("ms_recheck", ctypes.c_double), ("ms_cc", ctypes.c_double),
                ("ms_edges", ctypes.c_double), ("n_slots", ctypes.c_int64),
                ("pairs", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("band_pairs", ctypes.c_int64), ("bitmask_bytes", ctypes.c_int64),
                ("arena_peak_bytes", ctypes.c_uint64), ("precision", ctypes.c_int32),
                ("tile_m", ctypes.c_int32), ("tile_n", ctypes.c_int32),
                ("split_terms", ctypes.c_int32), ("tile_launches", ctypes.c_int32),
                ("band_halfwidth", ctypes.c_double),
                ("reserved_bytes", ctypes.c_uint64), ("reserve_overflow_bytes", ctypes.c_uint64),
                ("admission_waits", ctypes.c_int32), ("tile_passes_redone", ctypes.c_int32),
                ("tiles_screened_out", ctypes.c_int64), ("pairs_computed", ctypes.c_int64),
                ("tune_sampled", ctypes.c_int32), ("tune_pad", ctypes.c_int32),
                ("tune_pred_ms", ctypes.c_double * 5)]

    def as_dict(self) -> Dict:
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["tune_pred_ms"] = list(self.tune_pred_ms)
        return d


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_lib = None

EXPORTS = {
    "mapper_context_create": ([ctypes.c_int, _vp, ctypes.c_uint64, _vp, _P(_vp)], ctypes.c_int),
    "mapper_context_set_streams": ([_vp, _P(_vp), ctypes.c_int], ctypes.c_int),
    "mapper_context_destroy": ([_vp], None),
    "mapper_last_error": ([], ctypes.c_char_p),
    "mapper_context_memory": ([_vp, _P(ctypes.c_uint64), _P(ctypes.c_uint64)], ctypes.c_int),
    "mapper_cloud_create": ([_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _P(_vp)],
                            ctypes.c_int),
    "mapper_cloud_destroy": ([_vp], ctypes.c_int),
    "mapper_run": ([_vp, _vp, _P(_Params), _P(_vp)], ctypes.c_int),
    "mapper_knn_d2": ([_vp, _vp, ctypes.c_int32, ctypes.c_int32, _P(ctypes.c_double), _P(RunStats)],
                      ctypes.c_int),
    "mapper_run_eps_sweep": ([_vp, _vp, _P(_Params), _P(ctypes.c_double), ctypes.c_int32, _P(_vp)],
                             ctypes.c_int),
    "mapper_run_sweep": ([_vp, _vp, _P(_Params), _P(ctypes.c_double), ctypes.c_int32, _P(ctypes.c_int32),
                          ctypes.c_int32, _P(_vp)], ctypes.c_int),
    "mapper_submit": ([_vp, _vp, _P(_Params), _P(ctypes.c_uint64)], ctypes.c_int),
    "mapper_wait": ([_vp, ctypes.c_uint64, ctypes.c_int64, _P(_vp)], ctypes.c_int),
    "mapper_graph_num_nodes": ([_vp], ctypes.c_int64),
    "mapper_graph_num_edges": ([_vp], ctypes.c_int64),
    "mapper_graph_node_element": ([_vp], _P(ctypes.c_int32)),
    "mapper_graph_node_offsets": ([_vp], _P(ctypes.c_int64)),
    "mapper_graph_node_members": ([_vp], _P(ctypes.c_int32)),
    "mapper_graph_edges": ([_vp], _P(ctypes.c_int32)),
    "mapper_graph_edge_weights": ([_vp], _P(ctypes.c_int32)),
    "mapper_graph_stats": ([_vp, _P(RunStats)], ctypes.c_int),
    "mapper_graph_stage": ([_vp, ctypes.c_char_p, _P(ctypes.c_int64)], _vp),
    "mapper_graph_destroy": ([_vp], None),
    "mapper_debug_tile_d2": ([_vp, _vp, _P(ctypes.c_int32), ctypes.c_int32, ctypes.c_int32,
                              ctypes.c_double, _P(ctypes.c_double), _P(ctypes.c_double)],
                             ctypes.c_int),
    "mapper_debug_lens": ([_vp, _vp, _vp, _P(ctypes.c_double)], ctypes.c_int),
    "mapper_knn_d2_noalloc": ([_vp, _vp, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _vp],
                              ctypes.c_int),
    "mapper_debug_sqrt": ([_vp, _P(ctypes.c_double), ctypes.c_int64, _P(ctypes.c_double)], ctypes.c_int),
}


def load_library(path: str = LIB_PATH):
    """Load libmapper_gpu.so and declare every exported entry point."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() "
                          "(the mapper has no CPU fallback)")
    L = ctypes.CDLL(path)
    for name, (args, res) in EXPORTS.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(rc: int):
    if rc != MAPPER_OK:
        raise MapperError(rc, load_library().mapper_last_error().decode())


def _fptr(a: np.ndarray):
    return a.ctypes.data_as(_P(ctypes.c_float))


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(_P(ctypes.c_double))


def _check_axes(params, n: int, d: int):
    """The C ABI reads d direction floats and n lens values: check the sizes here."""
    for ax in params.axes:
        if ax.direction is not None and np.asarray(ax.direction).size != d:
            raise ValueError(f"projection direction has {np.asarray(ax.direction).size} values, cloud d = {d}")
        if ax.values is not None and np.asarray(ax.values).size != n:
            raise ValueError(f"lens values have {np.asarray(ax.values).size} entries, cloud n = {n}")


def make_params(params, flags: int = 0, keep: Optional[list] = None) -> _Params:
    """C struct for a synth.Params-like object (axes, eps, min_pts, precision)."""
    if keep is None:
        keep = []
    p = _Params()
    p.n_axes = len(params.axes)
    for a, ax in enumerate(params.axes):
        p.axis[a].kind = int(ax.kind)
        p.axis[a].column = int(ax.column)
        p.axis[a].n_intervals = int(ax.n_intervals)
        p.axis[a].overlap = float(ax.overlap)
        p.axis[a].cover = int(getattr(ax, "cover", 0))
        if ax.direction is not None:
            v = np.ascontiguousarray(ax.direction, dtype=np.float32)
            keep.append(v)
            p.axis[a].direction = _fptr(v)
        if ax.values is not None:
            v = np.ascontiguousarray(ax.values, dtype=np.float64)
            keep.append(v)
            p.axis[a].values = _dptr(v)
    p.eps = float(params.eps)
    p.min_pts = int(params.min_pts)
    p.precision = int(params.precision)
    p.flags = flags
    keep.append(p)
    return p


@dataclasses.dataclass
class Graph:
    node_element: np.ndarray
    node_offsets: np.ndarray
    node_members: np.ndarray
    edges: np.ndarray          # (E, 2) int32
    edge_weights: np.ndarray
    stats: Dict
    stages: Dict[str, np.ndarray]

    @property
    def n_nodes(self) -> int:
        return int(self.node_element.shape[0])

    @property
    def n_edges(self) -> int:
        return int(self.edges.shape[0])


_STAGES = {"lens": np.float64, "lo": np.float64, "hi": np.float64, "elem_offsets": np.int64,
           "elem_members": np.int32, "slot_count": np.int32, "slot_core": np.uint8,
           "slot_node": np.int32}


def _arr(ptr, count, dtype):
    if count <= 0 or not ptr:
        return np.zeros(0, dtype)
    buf = (ctypes.c_char * (int(count) * np.dtype(dtype).itemsize)).from_address(
        ctypes.cast(ptr, ctypes.c_void_p).value)
    return np.frombuffer(buf, dtype=dtype).copy()


def _take_graph(gp) -> Graph:
    L = load_library()
    try:
        nn = L.mapper_graph_num_nodes(gp)
        ne = L.mapper_graph_num_edges(gp)
        off = _arr(L.mapper_graph_node_offsets(gp), nn + 1, np.int64)
        st = RunStats()
        _check(L.mapper_graph_stats(gp, ctypes.byref(st)))
        stages = {}
        for name, dt in _STAGES.items():
            cnt = ctypes.c_int64(0)
            ptr = L.mapper_graph_stage(gp, name.encode(), ctypes.byref(cnt))
            if ptr:
                stages[name] = _arr(ptr, cnt.value, dt)
        return Graph(node_element=_arr(L.mapper_graph_node_element(gp), nn, np.int32),
                     node_offsets=off,
                     node_members=_arr(L.mapper_graph_node_members(gp), int(off[-1]) if nn else 0,
                                       np.int32),
                     edges=_arr(L.mapper_graph_edges(gp), 2 * ne, np.int32).reshape(ne, 2),
                     edge_weights=_arr(L.mapper_graph_edge_weights(gp), ne, np.int32),
                     stats=st.as_dict(), stages=stages)
    finally:
        L.mapper_graph_destroy(gp)


class Context:
    """A device arena (a torch uint8 tensor) plus a HIP stream."""

    def __init__(self, arena_bytes: int = 8 << 30, device: int = 0, stream=None,
                 serving_streams: int = 0):
        import torch
        self._torch = torch
        self.L = load_library()
        self.device = device
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=f"cuda:{device}")
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        h = _vp()
        _check(self.L.mapper_context_create(device, _vp(self.arena.data_ptr()), int(arena_bytes),
                                            _vp(self.stream.cuda_stream), ctypes.byref(h)))
        self.h = h
        self.slot_streams = []
        if serving_streams > 0:
            self.slot_streams = [torch.cuda.Stream(device=device) for _ in range(serving_streams)]
            arr = (_vp * serving_streams)(*[_vp(s.cuda_stream) for s in self.slot_streams])
            _check(self.L.mapper_context_set_streams(self.h, arr, serving_streams))

    def close(self):
        if getattr(self, "h", None):
            self.L.mapper_context_destroy(self.h)
            self.h = None
            self.arena = None          # the library no longer uses it: torch may reuse the memory

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def memory(self):
        a, b = ctypes.c_uint64(0), ctypes.c_uint64(0)
        _check(self.L.mapper_context_memory(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value

    def cloud(self, X) -> "Cloud":
        return Cloud(self, X)

    def knn_d2_noalloc(self, points, k: int, out, precision: int = 5):
        """k-NN squared distances of a device tensor of points (n x d FP32,
        contiguous) into the device tensor out (n float64), through the
        entry point that allocates nothing."""
        torch = self._torch
        if not (isinstance(points, torch.Tensor) and points.is_cuda and points.dtype == torch.float32
                and points.dim() == 2 and points.is_contiguous()):
            raise ValueError("points must be a contiguous n x d float32 CUDA tensor")
        n, d = points.shape
        if not (isinstance(out, torch.Tensor) and out.is_cuda and out.dtype == torch.float64
                and out.is_contiguous() and out.numel() == n):
            raise ValueError("out must be a contiguous float64 CUDA tensor of n elements")
        _check(self.L.mapper_knn_d2_noalloc(self.h, _vp(points.data_ptr()), int(n), int(d), int(k),
                                            int(precision), _vp(out.data_ptr())))
        return out

    def debug_sqrt(self, x) -> np.ndarray:
        """The library's FP64 square root kernel applied to host doubles."""
        a = np.ascontiguousarray(x, dtype=np.float64)
        out = np.empty_like(a)
        _check(self.L.mapper_debug_sqrt(self.h, _dptr(a), int(a.size), _dptr(out)))
        return out


class Cloud:
    """A point cloud resident in the context's arena."""

    def __init__(self, ctx: Context, X):
        self.ctx = ctx
        torch = ctx._torch
        if isinstance(X, torch.Tensor):
            T = X.detach().to(device=f"cuda:{ctx.device}", dtype=torch.float32).contiguous()
            n, d = T.shape
            ptr, on_dev, self._keep = T.data_ptr(), 1, T
        else:
            A = np.ascontiguousarray(X, dtype=np.float32)
            n, d = A.shape
            ptr, on_dev, self._keep = A.ctypes.data, 0, A
        self.n, self.d = int(n), int(d)
        h = _vp()
        _check(ctx.L.mapper_cloud_create(ctx.h, _vp(ptr), self.n, self.d, on_dev, ctypes.byref(h)))
        ctx.stream.synchronize()
        self._keep = None
        self.h = h

    def destroy(self):
        if self.h:
            _check(self.ctx.L.mapper_cloud_destroy(self.h))
            self.h = None

    def run(self, params, debug: bool = False, flags: int = 0) -> Graph:
        _check_axes(params, self.n, self.d)
        keep: list = []
        p = make_params(params, flags | (FLAG_DEBUG_STAGES if debug else 0), keep)
        g = _vp()
        _check(self.ctx.L.mapper_run(self.ctx.h, self.h, ctypes.byref(p), ctypes.byref(g)))
        return _take_graph(g)

    def run_eps_sweep(self, params, eps_list, debug: bool = False) -> List[Graph]:
        """The graphs for several eps values (at most MAX_EPS_VALUES) from one
        pass: graph t equals run(params with eps = eps_list[t])."""
        _check_axes(params, self.n, self.d)
        keep: list = []
        p = make_params(params, FLAG_DEBUG_STAGES if debug else 0, keep)
        eps = (ctypes.c_double * len(eps_list))(*[float(e) for e in eps_list])
        out = (_vp * len(eps_list))()
        _check(self.ctx.L.mapper_run_eps_sweep(self.ctx.h, self.h, ctypes.byref(p), eps, len(eps_list), out))
        return [_take_graph(_vp(out[t])) for t in range(len(eps_list))]

    def run_sweep(self, params, eps_list, minpts_list, debug: bool = False) -> List[List[Graph]]:
        """The graphs for every (eps, minPts) pair (at most MAX_EPS_VALUES eps
        and MAX_MINPTS_VALUES minPts values) from one pass: result[t][u]
        equals run(params with eps = eps_list[t], min_pts = minpts_list[u])."""
        _check_axes(params, self.n, self.d)
        keep: list = []
        p = make_params(params, FLAG_DEBUG_STAGES if debug else 0, keep)
        ne, nm = len(eps_list), len(minpts_list)
        eps = (ctypes.c_double * ne)(*[float(e) for e in eps_list])
        mps = (ctypes.c_int32 * nm)(*[int(m) for m in minpts_list])
        out = (_vp * (ne * nm))()
        _check(self.ctx.L.mapper_run_sweep(self.ctx.h, self.h, ctypes.byref(p), eps, ne, mps, nm, out))
        return [[_take_graph(_vp(out[t * nm + u])) for u in range(nm)] for t in range(ne)]

    def knn_d2(self, k: int, precision: int = 5):
        """k-th smallest canonical squared distance from every point to the
        others (exact); returns (values, stats dict)."""
        out = np.zeros(self.n, np.float64)
        st = RunStats()
        _check(self.ctx.L.mapper_knn_d2(self.ctx.h, self.h, int(k), int(precision),
                                        out.ctypes.data_as(_P(ctypes.c_double)), ctypes.byref(st)))
        return out, st.as_dict()

    def submit(self, params, debug: bool = False) -> int:
        _check_axes(params, self.n, self.d)
        keep: list = []
        p = make_params(params, FLAG_DEBUG_STAGES if debug else 0, keep)
        t = ctypes.c_uint64(0)
        _check(self.ctx.L.mapper_submit(self.ctx.h, self.h, ctypes.byref(p), ctypes.byref(t)))
        return int(t.value)

    def debug_lens(self, axis) -> np.ndarray:
        """Lens values of one axis (synth.Axis) computed on the GPU, host FP64."""
        from . import synth
        params = synth.Params([axis], eps=0.0, min_pts=1)
        _check_axes(params, self.n, self.d)
        keep: list = []
        p = make_params(params, 0, keep)
        out = np.empty(self.n, np.float64)
        _check(self.ctx.L.mapper_debug_lens(self.ctx.h, self.h, _vp(ctypes.addressof(p.axis[0])), _dptr(out)))
        return out

    def tile_d2(self, rows: Sequence[int], precision: int, eps: float):
        r = np.ascontiguousarray(rows, dtype=np.int32)
        m = r.shape[0]
        d2 = np.zeros((m, m), np.float64)
        band = np.zeros((m, m), np.float64)
        _check(self.ctx.L.mapper_debug_tile_d2(self.ctx.h, self.h, r.ctypes.data_as(_P(ctypes.c_int32)),
                                               m, int(precision), float(eps), _dptr(d2), _dptr(band)))
        return d2, band


def wait(ctx: Context, ticket: int, timeout_us: int = -1) -> Graph:
    g = _vp()
    _check(ctx.L.mapper_wait(ctx.h, ticket, int(timeout_us), ctypes.byref(g)))
    return _take_graph(g)
