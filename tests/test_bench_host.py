"""Host logic of bench.py (no GPU): the one-GPU contract and the roofline
entry computed from per-kernel HIP-event totals."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_roofline_takes_the_kernel_with_most_time(monkeypatch):
    monkeypatch.setattr(bench, "measured_traffic", lambda name: None)
    prof = {
        "relax0_f": {"launches": 4, "total_ms": 0.12, "bytes": 4 * 75e6, "avg_us": 30.0},
        "spmv0": {"launches": 2, "total_ms": 0.05, "bytes": 2 * 90e6, "avg_us": 25.0},
    }
    r = bench.roofline(prof, "c3", 2, 3, 24576)
    assert r["kernel"] == "relax0_f" and r["bound"] == "hbm" and r["unit"] == "GB/s"
    # algorithmic bytes per launch over the mean launch duration
    assert r["bytes_per_launch"] == 75e6
    assert r["achieved"] == pytest.approx(75e6 / 30e-6 / 1e9)
    assert r["peak"] == 8000.0
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["traffic"] is None


def test_roofline_traffic_is_keyed_by_workload(monkeypatch):
    seen = []
    monkeypatch.setattr(bench, "measured_traffic", lambda key: seen.append(key) or 123.0)
    prof = {"arnoldi_dot": {"launches": 3, "total_ms": 3.0, "bytes": 3 * 9e9, "avg_us": 1000.0}}
    r = bench.roofline(prof, "c3", 1, 3, 10)
    assert seen == ["c3:arnoldi_dot"] and r["traffic"] == 123.0
    assert r["achieved"] == pytest.approx(9e9 / 1e-3 / 1e9)
