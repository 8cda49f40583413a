"""Host logic of bench.py (no GPU): the single-GPU exit, the gating of the measured traffic
on the digest of the forward kernel's sources, and the algorithmic byte count of a launch."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stdout + r.stderr


def test_traffic_is_reported_only_for_the_profiled_sources(tmp_path, monkeypatch):
    good = tmp_path / "good.txt"
    good.write_text("# counters\nsource_sha256 = %s\ntraffic_bytes_per_launch = 1.5e+12\n"
                    % bench.kernel_source_digest())
    stale = tmp_path / "stale.txt"
    stale.write_text("source_sha256 = %s\ntraffic_bytes_per_launch = 1.5e+12\n" % ("0" * 64))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(good))
    assert bench.measured_traffic() == pytest.approx(1.5e12)
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(stale))
    assert bench.measured_traffic() is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(tmp_path / "missing.txt"))
    assert bench.measured_traffic() is None


def test_algorithmic_bytes_of_the_64_grid_launch():
    """8192 nodes of 33^3 points at K = 60 in FP32: 4 n (3K + K(K+1)/2) bytes each, the
    figure the roofline divides by the launch time."""
    n, K = 33 ** 3, 60
    assert bench.alg_bytes(n, K) == 4 * n * (3 * K + K * (K + 1) // 2)
    assert 8192 * bench.alg_bytes(n, K) == 2366943068160
