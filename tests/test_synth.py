"""The seeded input recipe (no GPU)."""
import numpy as np
import pytest

from paper_1907_02604_amd import synth


def test_hcp_site_counts():
    for L, count in [(8.0, 6), (24.0, 100), (32.0, 255), (48.0, 760), (64.0, 1925)]:
        assert synth.hcp_sites((L, L, L)).shape == (count, 3)


@pytest.mark.parametrize("cfg,n_atoms,nq", [(1, 6, 4096), (2, 255, 8192), (4, 16, 110592)])
def test_config_shapes(cfg, n_atoms, nq):
    P = synth.make_problem(cfg)
    assert P.atoms.shape == (n_atoms, 3)
    assert P.n_nodes == nq
    assert np.unique(P.centers).size == nq
    assert np.all((P.atoms >= 0) & (P.atoms < np.array(P.L)))
    assert P.v_loc.shape == P.n[::-1]
    assert P.v_loc.max() <= 0.0 and P.v_loc.min() > -10.0


def test_uneven_config_distributions():
    P = synth.make_problem(3, n_nodes=4000)
    assert set(np.unique(P.half_width)) == set(range(12, 25, 2))
    assert P.depth.min() >= 40 and P.depth.max() <= 100
    P5 = synth.make_problem(5, n_nodes=512, grid=64)
    assert np.all(P5.depth == 80)
    assert np.all(P5.weight == 64 ** 3 / 65536)


def test_seeded_determinism():
    a = synth.make_problem(2, n_nodes=64, grid=32)
    b = synth.make_problem(2, n_nodes=64, grid=32)
    assert np.array_equal(a.centers, b.centers)
    assert np.array_equal(a.atoms, b.atoms)
    assert np.array_equal(a.v_loc, b.v_loc)


def test_vloc_is_sum_of_gaussians():
    """One atom on a big grid: V at grid points equals depth*exp(-r^2/2sigma^2)."""
    N, h = 40, 0.5
    atom = np.array([[10.3, 9.6, 10.1]])
    V = synth.gaussian_vloc((N,) * 3, h, atom)
    for (ix, iy, iz) in [(20, 19, 20), (25, 17, 22), (10, 30, 15)]:
        r2 = np.sum((np.array([ix, iy, iz]) * h - atom[0]) ** 2)
        ref = -2.0 * np.exp(-r2 / 2.0) if r2 <= 64.0 else 0.0
        assert V[iz, iy, ix] == pytest.approx(ref, abs=1e-15)


def test_screw_displacement():
    L = (64.0, 64.0, 64.0)
    s = np.array([[40.0, 32.0, 5.0], [32.0, 40.0, 5.0], [24.0, 32.0 - 1e-9, 5.0]])
    d = synth.screw_displace(s, L)
    np.testing.assert_allclose(d[:, 2] - 5.0, [0.0, 6.06 / 4, -6.06 / 2], atol=1e-8)


def test_coarse_esps_zone_and_sample():
    """The full-resolution zone holds every point of the disk on every z plane; the
    seeded sample adds points; the result is sorted, unique and reproducible."""
    n = (20, 20, 6)
    a = synth.coarse_esps(n, 9, 50, 3)
    assert np.array_equal(a, synth.coarse_esps(n, 9, 50, 3))
    assert np.all(np.diff(a) > 0)
    disk = sum(1 for x in range(20) for y in range(20) if (x - 10) ** 2 + (y - 10) ** 2 <= 9)
    x, y, z = a % 20, (a // 20) % 20, a // 400
    in_zone = (x - 10) ** 2 + (y - 10) ** 2 <= 9
    assert disk == 29 and in_zone.sum() == 6 * disk
    assert disk * 6 < a.size <= disk * 6 + 50
