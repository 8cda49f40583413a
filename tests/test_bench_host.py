"""Host logic of bench.py (no GPU): the single-GPU exit, the gating of the measured traffic
on the digest of the forward kernel's sources, and the algorithmic byte count of a launch."""
import os
import subprocess
import sys

import numpy as np
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


def test_stratified_order_visits_every_stratum_in_each_round():
    """Every run of n_bins consecutive ids holds one node of each cost bin, so a prefix of
    any length is spread over the cost range; the order is a permutation and seeded."""
    import numpy as np
    cost = np.random.default_rng(3).uniform(size=103)
    order = bench.stratified_order(cost, 10, 7)
    assert sorted(order.tolist()) == list(range(103))
    bins = np.array_split(np.argsort(cost, kind="stable"), 10)
    which = {int(q): b for b, ids in enumerate(bins) for q in ids}
    for r in range(10):
        assert sorted(which[int(q)] for q in order[10 * r:10 * r + 10]) == list(range(10))
    assert np.array_equal(order, bench.stratified_order(cost, 10, 7))


def test_error_metrics():
    """Normwise error over the largest reference value, and the per-node relative error over
    the nodes above the floor only (a tiny reference value does not count)."""
    import numpy as np
    ref = np.array([1.0, 0.5, 1e-5, -0.2])
    got = ref + np.array([1e-6, -1e-6, 1e-6, 4e-6])
    e = bench.errors(got, ref)
    assert e["normwise_rel_err"] == pytest.approx(4e-6)
    assert e["per_node_rel_err_max"] == pytest.approx(2e-5)
    assert e["nodes_above_floor"] == 3


def test_cube_points_and_launch_bytes_of_an_untruncated_node():
    """Untruncated nodes cover the whole grid; FP64 storage doubles the bytes."""
    from paper_1907_02604_amd import synth
    P1 = synth.make_problem(1)
    assert np.all(bench.cube_points(P1.half_width, P1.n) == 16 ** 3)
    assert bench.launch_bytes(P1, elem=8) == pytest.approx(4096 * 8 * 4096 * (90 + 465))
