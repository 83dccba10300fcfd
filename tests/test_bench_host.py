"""Host-side logic of bench.py (CPU only): the one-GPU guard, the work per pair
behind the roofline, and how HBM traffic is taken from a counters summary only
when it was measured on the current kernel source."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused_before_touching_a_device():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and not r.stdout


def test_work_per_pair():
    # paper's form: 42 FMA-class operations and M + 1 = 11 transcendentals
    assert bench.pair_work(3.5) == pytest.approx(80.5)
    assert bench.pair_work(1.0, M=4) == pytest.approx(47.0)
    # implemented polynomial form: 44 operations and one reciprocal square root
    assert bench.pair_work_implemented(3.5) == pytest.approx(47.5)
    assert bench.mode_work(3.5) == pytest.approx((13.0, 16.0))
    assert bench.VALU_LANE_OPS_PER_S == pytest.approx(78.6432e12)


def test_traffic_only_from_counters_of_the_current_kernel(tmp_path, monkeypatch):
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_hash", lambda: "0123456789abcdef")
    f = tmp_path / "profiles" / "pair_kernel_slab-1m_counters.txt"
    assert bench.read_traffic("slab-1m") is None  # no summary
    f.write_text("# header: with a colon\nkernels_sha256: 0123456789abcdef\nhbm_bytes_per_launch: 1.6575e+08\n")
    assert bench.read_traffic("slab-1m") == pytest.approx(1.6575e8)
    f.write_text("kernels_sha256: fedcba9876543210\nhbm_bytes_per_launch: 1.6575e+08\n")
    assert bench.read_traffic("slab-1m") is None  # taken on another kernel source
    f.write_text("kernels_sha256: 0123456789abcdef\n")
    assert bench.read_traffic("slab-1m") is None  # no traffic figure
