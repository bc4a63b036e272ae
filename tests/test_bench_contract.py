"""bench.py's host logic on the CPU: the roofline arithmetic, the traffic
figure's gate on the kernel source, and the one-GPU contract."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_roofline_from_launch_totals():
    """achieved = algorithmic bytes over event time; averages per launch.
    Without per-step model bytes the algorithmic bytes are the launch's own."""
    r = bench.roofline_of((1000, 250.0, 2.0e12), "k", traffic=3.0e9)
    assert r["achieved"] == pytest.approx(8000.0)          # 2e12 B in 0.25 s
    assert r["frac"] == pytest.approx(1.0)
    assert r["avg_launch_us"] == pytest.approx(250.0)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(2.0e9)
    assert r["achieved_minimal"] == pytest.approx(8000.0)
    assert r["traffic"] == 3.0e9 and r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["achieved_hbm_counters"] == pytest.approx(12000.0)   # 3e9 B per 250 us launch
    empty = bench.roofline_of((0, 0.0, 0.0), "k")
    assert empty["achieved"] is None and empty["avg_launch_us"] is None


def test_roofline_counts_the_per_step_model():
    """A smoother kind carries both byte counts: achieved follows the per-step
    model (each fused sweep, residual and correction counted as its own pass),
    the minimal count (every value once) is reported beside it."""
    r = bench.roofline_of((100, 50.0, 1.0e11, 3.0e11), "k")
    assert r["achieved"] == pytest.approx(6000.0)          # 3e11 B in 0.05 s
    assert r["frac"] == pytest.approx(0.75)
    assert r["algorithmic_bytes_per_launch"] == pytest.approx(3.0e9)
    assert r["achieved_minimal"] == pytest.approx(2000.0)
    assert r["frac_minimal"] == pytest.approx(0.25)
    assert r["minimal_bytes_per_launch"] == pytest.approx(1.0e9)


def test_traffic_is_dropped_when_the_kernel_source_changed(tmp_path):
    digest = bench.kernel_source_digest()
    assert len(digest) == 16 and int(digest, 16) >= 0
    good = tmp_path / "t.md"
    good.write_text(f"- hbm_bytes_per_launch: `1.5e8`\n- kernel_source_sha256: `{digest}`\n")
    assert bench.read_traffic(str(good)) == pytest.approx(1.5e8)
    stale = tmp_path / "s.md"
    stale.write_text("- hbm_bytes_per_launch: `1.5e8`\n- kernel_source_sha256: `0000000000000000`\n")
    assert bench.read_traffic(str(stale)) is None
    assert bench.read_traffic(str(tmp_path / "missing.md")) is None


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stdout
