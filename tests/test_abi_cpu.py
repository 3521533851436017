"""The C-ABI library, without a GPU: it loads, it exports every entry point that
include/mapper_gpu.h declares, and its errors are reported through return codes."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mapper_gpu.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(mapper_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("mapper_context_create", "mapper_cloud_create", "mapper_run", "mapper_submit",
                 "mapper_wait", "mapper_graph_edges", "mapper_debug_tile_d2"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2011_03209_amd import binding
    L = binding.load_library()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    # the binding declares argument types for exactly the header's functions
    assert sorted(binding.EXPORTS) == declared_functions()


def test_errors_without_a_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2011_03209_amd import binding
    L = binding.load_library()
    h = ctypes.c_void_p()
    # misaligned / tiny arena -> EINVAL before touching the device
    rc = L.mapper_context_create(0, ctypes.c_void_p(4096 + 8), 1 << 30, None, ctypes.byref(h))
    assert rc == binding.MAPPER_EINVAL
    assert b"aligned" in L.mapper_last_error()
    rc = L.mapper_context_create(0, ctypes.c_void_p(4096), 1 << 30, None, ctypes.byref(h))
    assert rc == binding.MAPPER_EDEVICE
    # null arguments are rejected, not dereferenced
    assert L.mapper_run(None, None, None, ctypes.byref(h)) == binding.MAPPER_EINVAL
    assert L.mapper_run_eps_sweep(None, None, None, None, 2, ctypes.byref(h)) == binding.MAPPER_EINVAL
    assert L.mapper_run_sweep(None, None, None, None, 2, None, 2, ctypes.byref(h)) == binding.MAPPER_EINVAL
    assert L.mapper_knn_d2(None, None, 3, 2, None, None) == binding.MAPPER_EINVAL
    assert L.mapper_graph_num_nodes(None) == 0
