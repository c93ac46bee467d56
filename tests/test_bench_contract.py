"""bench.py's host-side contract (CPU): one GPU only, and the roofline
arithmetic of its JSON line."""
from __future__ import annotations

import os
import subprocess
import sys
import types

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_with_a_message():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout == ""


def test_roofline_is_algorithmic_bytes_over_the_average_launch():
    n = 512
    cells = n**3
    # two reports: 10 + 8 timed launches over 9.0 + 7.2 ms -> 0.9 ms per launch
    reps = [types.SimpleNamespace(smooth_launches=10, t_smooth_ms=9.0,
                                  smooth_cells_per_launch=cells),
            types.SimpleNamespace(smooth_launches=8, t_smooth_ms=7.2,
                                  smooth_cells_per_launch=cells)]
    r = bench.roofline(reps, n, copy_gbs=5600.0)
    alg = bench.BYTES_PER_UPDATE_FP64 * cells
    assert r["alg_bytes_per_launch"] == alg
    assert r["avg_launch_us"] == pytest.approx(900.0)
    assert r["achieved"] == pytest.approx(alg / 0.9e-3 / 1e9, abs=0.05)
    assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS, abs=1e-4)
    assert r["frac_of_copy"] == pytest.approx(r["achieved"] / 5600.0, abs=1e-4)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0


def test_no_timed_launches_give_no_roofline():
    reps = [types.SimpleNamespace(smooth_launches=0, t_smooth_ms=0.0,
                                  smooth_cells_per_launch=0)]
    assert bench.roofline(reps, 512) is None


def test_traffic_is_taken_only_for_the_kernels_it_was_measured_on(tmp_path, monkeypatch):
    """The HBM bytes of the profiles count only while the kernel sources hash
    to the value stored with them."""
    h = bench.kernel_source_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "smoother_traffic.json").write_text(
        '{"kernel_hash": "%s", "bytes_per_launch": {"512": 3.9e9}}' % h)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.traffic_from_profiles(512) == pytest.approx(3.9e9)
    assert bench.traffic_from_profiles(256) is None
    (prof / "smoother_traffic.json").write_text(
        '{"kernel_hash": "0000000000000000", "bytes_per_launch": {"512": 3.9e9}}')
    assert bench.traffic_from_profiles(512) is None
