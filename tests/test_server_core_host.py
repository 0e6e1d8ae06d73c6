"""Sanitizer builds of the library's host-side logic, run on the CPU.

* tests/server_core_check.cpp drives the solve server's HBM ledger and its
  ticket book (server_core.hpp; the code wd_server_* runs) under the address
  and undefined-behaviour sanitizers, and again under the thread sanitizer
  with client threads submitting and polling while a scheduler thread
  publishes.
* tests/layout_check.cpp (site order, neighbours, launch shapes, partial-sum
  capacity) under the address and undefined-behaviour sanitizers.

Both are plain g++ builds of host code: no HIP device code is compiled.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_04201_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def _build_run(tmp_path, src, sanitize, extra=(), timeout=300):
    exe = tmp_path / ("check_" + sanitize.replace(",", "_"))
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=" + sanitize, "-fno-sanitize-recover=all", *extra,
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, src, "-o", str(exe), "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=timeout, env=env)
    assert out.returncode == 0 and out.stdout.strip().endswith("OK"), out.stdout + out.stderr
    return out.stdout


@pytest.mark.parametrize("sanitize", ["address,undefined", "thread"])
def test_server_core_sanitized(tmp_path, sanitize):
    _build_run(tmp_path, os.path.join(ROOT, "tests", "server_core_check.cpp"), sanitize)


def test_layout_check_sanitized(tmp_path):
    hip_inc = "/opt/rocm/include"
    if not os.path.isdir(hip_inc):
        pytest.skip("HIP headers not available")
    _build_run(tmp_path, os.path.join(ROOT, "tests", "layout_check.cpp"), "address,undefined",
               extra=("-D__HIP_PLATFORM_AMD__", "-I", hip_inc))
