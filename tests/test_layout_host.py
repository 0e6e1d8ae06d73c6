"""Host test of the library's internal site order and neighbour arithmetic:
compiles tests/layout_check.cpp against the library's internal header and
runs it on the CPU (every brick shape of several lattices, brute force)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_layout_and_neighbours(tmp_path):
    exe = tmp_path / "layout_check"
    src = os.path.join(ROOT, "tests", "layout_check.cpp")
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_1810_04201_amd", "csrc"), src, "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "hipcc" in (r.stderr or "") and not os.path.exists("/opt/rocm"):
        pytest.skip("hipcc not available")
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout
