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
