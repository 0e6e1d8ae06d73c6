"""Host tests of bench.py's contract and of its counter arithmetic (no GPU):
--gpus above 1 exits with a message, and the traffic summary scales
FETCH_SIZE / WRITE_SIZE by the calibration copy and matches the stencil
kernels whatever their scheduling-group template argument."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")
V = 48 * 48 * 48 * 96
COPY = 256 * 1024 * 1024 * 8  # the probe's calibration copy, bytes read and written


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Grid_Size", "Counter_Name",
                               "Counter_Value"])
        w.writeheader()
        for i, (name, grid, kib) in enumerate(rows):
            w.writerow({"Dispatch_Id": i + 1, "Kernel_Name": name, "Grid_Size": grid,
                        "Counter_Name": counter, "Counter_Value": kib})


@pytest.mark.parametrize("group", [1, 3])
def test_pmc_summary_scales_and_matches_kernels(tmp_path, group):
    plain = f"void wd::k_dslash_tm<0, false, false, {group}, false, false, 3>(wd::Geom, ...)"
    xr = f"void wd::k_dslash_tm<0, true, true, {group}, false, true, 3>(wd::Geom, ...)"
    halo = f"void wd::k_dslash_tm<0, false, false, {group}, true, false, 3>(wd::Geom, ...)"
    # the copy counters read half the bytes on fetch (64-byte accounting of
    # 128-byte reads) and all of them on write; a small status-word copy runs too
    fetch = [("__amd_rocclr_copyBuffer", 8, 1.0),
             ("__amd_rocclr_copyBuffer", 1 << 20, COPY / 2 / 1024),
             (plain, 4608, 5.0e6), (plain, 4608, 5.0e6), (halo, 999, 1.0),
             (xr, 4608, 6.0e6), (xr, 4608, 10.0)]  # a gated no-op launch
    write = [("__amd_rocclr_copyBuffer", 8, 1.0),
             ("__amd_rocclr_copyBuffer", 1 << 20, COPY / 1024),
             (plain, 4608, 2.0e6), (plain, 4608, 2.0e6), (halo, 999, 1.0),
             (xr, 4608, 2.0e6), (xr, 4608, 0.0)]
    fc, wc, out = tmp_path / "f.csv", tmp_path / "w.csv", tmp_path / "t.json"
    _write(fc, "FETCH_SIZE", fetch)
    _write(wc, "WRITE_SIZE", write)
    r = subprocess.run([sys.executable, BENCH, "--pmc-summary", str(fc), str(wc), "--out",
                        str(out), "--cmd", "test"], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    t = json.load(open(out))
    assert t["copy_calibration"]["fetch_factor"] == 2.0
    assert t["copy_calibration"]["write_factor"] == 1.0
    k = t["kernels"]["dslash_f64"]
    assert k["traffic_bytes"] == round(5.0e6 * 1024 * 2 + 2.0e6 * 1024)
    assert k["algorithmic_bytes"] == V * 768  # 12-real links: 384 + 2 x 192
    assert k["traffic_bytes_per_site"] == round(k["traffic_bytes"] / V, 1)
    x = t["kernels"]["dslash_xr_f64"]  # the no-op launch is left out
    assert x["traffic_bytes"] == round(6.0e6 * 1024 * 2 + 2.0e6 * 1024)
    assert x["algorithmic_bytes"] == V * 960  # + r read and written
