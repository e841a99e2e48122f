"""Host-side pieces of bench.py: the roofline record built from a solve's
smoother counters, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _reps(seconds, nbytes, launches):
    return [{"smooth_seconds": seconds, "smooth_bytes": nbytes, "smooth_launches": launches}]


def test_roofline_from_counters():
    import bench
    # two solves: 100 launches of 12.29 MB in 1 ms of launch time in all
    reps = _reps(4e-4, 40 * 12.29e6, 40) + _reps(6e-4, 60 * 12.29e6, 60)
    r = bench.roofline(reps, traffic=31.6e6)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert r["launches"] == 100
    assert r["achieved"] == pytest.approx(100 * 12.29e6 / 1e-3 / 1e9)
    assert r["frac"] == pytest.approx(r["achieved"] / 8000.0)
    assert r["avg_launch_us"] == pytest.approx(10.0)
    assert r["alg_bytes_per_launch"] == pytest.approx(12.29e6)
    assert r["traffic"] == 31.6e6 and r["traffic_unit"].startswith("bytes per launch")


def test_roofline_without_row_kernel_sweeps():
    """A grid whose levels all run in the coarse-level kernel has no
    row-kernel sweep to price: no bandwidth figure is reported."""
    import bench
    r = bench.roofline(_reps(0.0, 0.0, 0))
    assert r["launches"] == 0
    assert r["achieved"] is None and r["frac"] is None
    assert r["bound"] == "latency"


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]
