"""The C ABI on the host: symbols, argument validation, the host Gauss-rule solver."""
import ctypes
import os
import re

import numpy as np
import pytest
import scipy.linalg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def sgq():
    from paper_1907_02604_amd import sgq as mod
    return mod


def _header_functions():
    src = open(os.path.join(ROOT, "include", "sgq.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char\*|void)\s+\**(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_function(sgq):
    names = _header_functions()
    assert "rho_quadrature" in names and "band_energy_backward" in names
    lib = ctypes.CDLL(sgq.LIB_PATH)
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(sgq.EXPORTED)


def test_validate_accepts_configs(sgq):
    assert sgq.validate((64, 64, 64), 0.5, 255, 4, [0, 5], [16, 16], [60, 60], sgq.SGQ_FP32) == 0
    assert sgq.validate((16, 16, 16), 0.5, 6, 0, [3], [-1], [30], sgq.SGQ_FP64) == 0
    assert sgq.validate((96,) * 3, 0.5, 760, 4, [1], [24], [100], sgq.SGQ_FP32) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(n=(0, 4, 4)), -1),
    (dict(h=0.0), -1),
    (dict(n_proj=3), -1),
    (dict(centers=[64 ** 3]), -1),
    (dict(centers=[-1]), -1),
    (dict(depth=[0]), -1),
    (dict(depth=[129]), -1),
    (dict(half_width=[29]), -1),     # 59 > 64 - 6
    (dict(half_width=[-2]), -1),
    (dict(precision=7), -1),
])
def test_validate_rejects(sgq, kw, code):
    args = dict(n=(64, 64, 64), h=0.5, n_atoms=10, n_proj=4, centers=[0], half_width=[16],
                depth=[60], precision=sgq.SGQ_FP32)
    args.update(kw)
    assert sgq.validate(**args) == code
    assert len(sgq.lib().sgq_last_error()) > 0


def test_validate_cube_limit_edge(sgq):
    # 2R+1 = 58 = 64 - 6 is the largest accepted cube
    assert sgq.validate((64,) * 3, 0.5, 1, 4, [0], [28], [10], sgq.SGQ_FP32) == 0
    assert sgq.validate((64,) * 3, 0.5, 1, 4, [0], [29], [10], sgq.SGQ_FP32) == -1


@pytest.mark.parametrize("K", [1, 2, 7, 60, 100, 128])
def test_host_gauss_rule_matches_lapack(sgq, K):
    rng = np.random.default_rng(K)
    a = rng.uniform(-2, 30, K)
    b = rng.uniform(0.05, 9, K - 1)
    if K > 10:
        b[3] = 1e-12          # nearly split matrix
    th, w = sgq.gauss_rule_host(a, b)
    if K == 1:
        ref_t, ref_w = a, np.ones(1)
    else:
        ref_t, S = scipy.linalg.eigh_tridiagonal(a, b)
        ref_w = S[0] ** 2
    np.testing.assert_allclose(th, ref_t, rtol=1e-13, atol=1e-12)
    np.testing.assert_allclose(w, ref_w, atol=1e-13)
    assert abs(w.sum() - 1) < 1e-13


def test_host_gauss_rule_rejects_bad_sizes(sgq):
    with pytest.raises(sgq.SgqError):
        sgq.gauss_rule_host(np.zeros(0), np.zeros(0))
    with pytest.raises(sgq.SgqError):
        sgq.gauss_rule_host(np.zeros(129), np.ones(128))


def test_fermi_level_rejects_bad_arguments_on_the_host():
    """Argument errors are returned before anything is launched (no plan needed)."""
    from paper_1907_02604_amd import sgq
    lib = sgq.lib()
    assert lib.sgq_fermi_level(None, None, None, 1.0, 0.01, 1e-12, None, None) == sgq.SGQ_EINVAL


def test_cluster_energy_rejects_bad_arguments_on_the_host():
    from paper_1907_02604_amd import sgq
    lib = sgq.lib()
    assert lib.sgq_cluster_energy(None, None, None, None, 1, 1, None, None, None, None) == sgq.SGQ_EINVAL


# ------------------------------------------------------------------ cluster geometry (host)
@pytest.mark.parametrize("n,radius", [((12, 10, 9), 0.0), ((12, 10, 9), 0.5), ((12, 10, 9), 0.71),
                                      ((12, 10, 9), 1.2), ((12, 10, 9), 3.0), ((7, 16, 5), 1.5)])
def test_cluster_build_matches_the_oracle_balls(sgq, n, radius):
    """Each cluster of the CSR list is the oracle's brute-force ball (periodic wrap
    included: a radius of 3 bohr reaches past half of a 9-point axis)."""
    import oracle as O
    h = 0.5
    rng = np.random.default_rng(3)
    c = rng.choice(int(np.prod(n)), 6, replace=False)
    c[1] = c[0] + 1 if (c[0] + 1) % n[0] else c[0] - 1      # two overlapping clusters
    out = sgq.cluster_build(n, h, c, radius, esp_weight=np.arange(1.0, 7.0))
    nc, off, mem = out["node_center"], out["member_offset"], out["member_node"]
    assert np.all(np.diff(nc) > 0)
    for q in range(c.size):
        ref = O.cluster_members(n, h, int(c[q]), radius)
        assert np.array_equal(nc[mem[off[q]:off[q + 1]]], ref)
    union = np.unique(np.concatenate([O.cluster_members(n, h, int(x), radius) for x in c]))
    assert np.array_equal(nc, union)
    # node_esp: the lowest cluster holding each node
    for k, p in enumerate(nc):
        holders = [q for q in range(c.size) if p in set(nc[mem[off[q]:off[q + 1]]].tolist())]
        assert out["node_esp"][k] == holders[0]
    # node weights carry sum_q n_q Fbar_q for any per-node energy
    e = rng.normal(size=nc.size)
    fbar = np.array([e[mem[off[q]:off[q + 1]]].mean() for q in range(c.size)])
    assert abs(np.dot(out["node_weight"], e) - np.dot(np.arange(1.0, 7.0), fbar)) < 1e-12


def test_cluster_build_reports_counts_and_capacity(sgq):
    lib = sgq.lib()
    dims = np.array([10, 10, 10], np.int32)
    c = np.array([0, 555], np.int64)
    nn, nm = ctypes.c_int64(0), ctypes.c_int64(0)
    args = (dims.ctypes.data, 0.5, c.ctypes.data, 2, 1.0, None)
    assert lib.sgq_cluster_build(*args, 0, 0, None, None, None, None, None,
                                 ctypes.byref(nn), ctypes.byref(nm)) == sgq.SGQ_OK
    assert (nn.value, nm.value) == (66, 66)       # two disjoint 33-point balls
    nodes = np.zeros(65, np.int64)
    assert lib.sgq_cluster_build(*args, 65, 66, nodes.ctypes.data, None, None, None, None,
                                 ctypes.byref(nn), ctypes.byref(nm)) == sgq.SGQ_EINVAL
    bad = (dims.ctypes.data, 0.5, c.ctypes.data, 2, -1.0, None)
    assert lib.sgq_cluster_build(*bad, 0, 0, None, None, None, None, None,
                                 ctypes.byref(nn), ctypes.byref(nm)) == sgq.SGQ_EINVAL
    outside = np.array([1000], np.int64)
    assert lib.sgq_cluster_build(dims.ctypes.data, 0.5, outside.ctypes.data, 1, 1.0, None, 0, 0,
                                 None, None, None, None, None, ctypes.byref(nn),
                                 ctypes.byref(nm)) == sgq.SGQ_EINVAL


def test_potential_and_fe_reject_bad_arguments_on_the_host(sgq):
    """Grid and mesh validation happens before any device call."""
    lib = sgq.lib()
    h = ctypes.c_void_p()
    for n, hh in (((7, 8, 8), 0.5), ((8, 8, 8), -1.0), ((2048, 1, 1), 0.5), ((0, 4, 4), 0.5)):
        dims = np.array(n, np.int32)
        assert lib.sgq_potential_create(dims.ctypes.data, hh, ctypes.byref(h)) == sgq.SGQ_EINVAL
    assert lib.sgq_lda_xc(None, -1, None, None, None) == sgq.SGQ_EINVAL
    assert lib.sgq_lda_xc(None, 0, None, None, None) == sgq.SGQ_OK
    dims = np.array([8, 8, 8], np.int32)
    esp = np.array([0, 7, 56, 448], np.int64)
    bad = np.array([[0, 1, 2, 4]], np.int32)
    assert lib.sgq_fe_mesh_create(dims.ctypes.data, esp.ctypes.data, 4, bad.ctypes.data, 1, 2,
                                  ctypes.byref(h)) == sgq.SGQ_EINVAL
    ok = np.array([[0, 1, 2, 3]], np.int32)
    assert lib.sgq_fe_mesh_create(dims.ctypes.data, esp.ctypes.data, 4, ok.ctypes.data, 1, 5,
                                  ctypes.byref(h)) == sgq.SGQ_EINVAL      # max_fields > 4
    big = np.array([70000, 2, 2], np.int32)
    assert lib.sgq_fe_mesh_create(big.ctypes.data, esp.ctypes.data, 4, ok.ctypes.data, 1, 2,
                                  ctypes.byref(h)) == sgq.SGQ_EINVAL


def test_plan_switches_reject_a_null_plan(sgq):
    lib = sgq.lib()
    assert lib.sgq_plan_set_retain(None, 1, 0, None) == sgq.SGQ_EINVAL
    assert lib.sgq_plan_set_graph(None, 1) == sgq.SGQ_EINVAL
    assert lib.sgq_plan_set_schedule(None, 0) == sgq.SGQ_EINVAL
