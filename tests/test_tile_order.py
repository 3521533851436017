"""The tile order of the distance-tile launch (host build of internal.h).

The tile launch, its item table and the components kernels all locate a tile
pair and its bitmask block through tile_decode / tile_local_index and the
host's supertile-column table.  tests/host/tile_order_check.cpp checks, for
every supertile size the runtime can choose and for multi-element tables with
ragged and empty elements, that the decode is one to one onto the pairs
I <= J < T of each element, that each item owns its own bitmask block, and
that tile_local_index inverts it.  It needs hipcc (for the HIP headers), not
a GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_tile_order_is_a_bijection(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc is not installed")
    exe = str(tmp_path / "tile_order_check")
    src = os.path.join(ROOT, "tests", "host", "tile_order_check.cpp")
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2011_03209_amd", "csrc"), src, "-o", exe],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([exe, "160"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
