"""Host-side logic of bench.py (no GPU): the single-GPU guard, the roofline
entry's arithmetic and the source-keyed traffic lookup."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    msg = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_roofline_entry_of_a_grid_kernel():
    k = {"name": "k_pre_s<double, 2, 32>", "avg_ms": 0.5, "bytes_per_launch": 2.0e9, "flops_per_launch": 1.0e9}
    row = bench.kernel_row(k, "f64")
    assert row["bound"] == "hbm" and row["unit"] == "GB/s"
    assert row["achieved"] == pytest.approx(4000.0)               # 2 GB in 0.5 ms
    assert row["frac"] == pytest.approx(4000.0 / bench.HBM_PEAK_GBS)


def test_roofline_entry_of_the_persistent_kernel():
    k = {"name": "k_subtree<double, 512, false>", "avg_ms": 0.016, "bytes_per_launch": 15376.0,
         "flops_per_launch": 262813.2}
    row = bench.kernel_row(k, "f64")
    ach = 262813.2 / 16e-6 / 1e12
    assert row["bound"] == "alu" and row["unit"] == "TFLOP/s" and row["peak"] == 78.6
    assert row["achieved"] == pytest.approx(ach, abs=1e-4)
    assert row["frac"] == pytest.approx(ach / 78.6, abs=1e-6)
    assert row["frac_of_one_cu"] == pytest.approx(ach / (78.6 / 256), abs=1e-4)


def test_traffic_lookup_is_keyed_by_the_kernel_source():
    with open(os.path.join(ROOT, "profiles", "traffic.json")) as fh:
        data = json.load(fh)
    with open(os.path.join(ROOT, "paper_2010_00626_amd", "csrc", "kc_kernels.hip"), "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()
    name = next(iter(data["bytes_per_launch"]))
    got = bench.traffic_of(name)
    if data["kernels_source_sha256"] == digest:
        assert got == round(data["bytes_per_launch"][name], 1)
    else:
        assert got is None
    assert bench.traffic_of("no such kernel") is None
