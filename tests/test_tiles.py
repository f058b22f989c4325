"""Host logic: the workgroup -> tile orders of the GEMM kernels (tiles.h).

tests/tiles_check.cpp is built with hipcc for the host and checks that the
XCD-aware order visits every output tile exactly once for 48 x 48 tile counts
and larger shapes, and that a diagonal pair batch's grid visits exactly the
kept tiles (those holding some pair with p <= q) once each, for batch sizes 1..40
and pair extents 2..602 with 128- and 64-wide tiles, and that the split-K order
on a one-dimensional grid takes every (K chunk, tile) once with all tiles of a
chunk on one XCD."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_tile_orders_are_bijections(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "tiles_check")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-O2", "-std=c++17", "-I",
                    os.path.join(ROOT, "paper_2401_11935_amd", "csrc"), os.path.join(HERE, "tiles_check.cpp"),
                    "-o", exe], check=True, capture_output=True, timeout=300)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout[-2000:]
    assert "tiles ok" in out.stdout
