"""Predictor + corrector reconstruction on the fine grid (sgq_fe_*) on the GPU against the
FP64 oracle: exact point location, interpolated fields, and the measured 128^3 workload."""
import numpy as np
import pytest

import oracle as O
from paper_1907_02604_amd import synth
from gpu_util import announce, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def _grid_xyz(n, idx=None):
    idx = np.arange(int(np.prod(n))) if idx is None else np.asarray(idx)
    return np.stack([idx % n[0], (idx // n[0]) % n[1], idx // (n[0] * n[1])], 1)


def _device_run(n, esp, tets, vals, pred, max_fields=None):
    import torch
    from paper_1907_02604_amd import sgq
    F = vals.shape[0]
    mesh = sgq.FeMesh(n, esp, tets, max_fields=max_fields or F)
    loc = torch.empty(int(np.prod(n)), dtype=torch.int32, device="cuda")
    mesh.location(loc)
    v = torch.as_tensor(np.ascontiguousarray(vals), device="cuda")
    p = torch.as_tensor(np.ascontiguousarray(pred.reshape(F, -1)), device="cuda")
    out = torch.empty_like(p)
    mesh.reconstruct(v, p, out)
    torch.cuda.synchronize()
    info = mesh.info()
    mesh.close()
    return loc.cpu().numpy(), out.cpu().numpy(), info


@pytest.mark.parametrize("seed,n,m,F", [(3, (14, 13, 12), 60, 2), (5, (20, 9, 16), 150, 1),
                                        (6, (17, 17, 17), 400, 3), (7, (9, 30, 11), 90, 4)])
def test_location_and_fields_match_oracle(seed, n, m, F):
    """Every grid point's tetrahedron equals the oracle's brute-force choice bit for bit; the
    fields agree to FP64 rounding (barycentric coordinates as volume ratios on the device,
    as a 4x4 solve in the oracle)."""
    rng = np.random.default_rng(seed)
    esp = np.sort(rng.choice(int(np.prod(n)), m, replace=False))
    tets = synth.esp_mesh(n, esp)
    pred = rng.normal(size=(F, int(np.prod(n))))
    vals = rng.normal(size=(F, m))
    announce(f"fe: {n} grid, {m} ESPs, {len(tets)} tets, {F} fields")
    loc, out, info = _device_run(n, esp, tets, vals, pred)
    ref_loc = O.fe_locate(n, esp, tets, _grid_xyz(n))
    assert np.array_equal(loc, ref_loc)
    assert info["kept"] == len(tets)
    ref = O.fe_reconstruct(n, esp, tets, vals, pred)
    err = np.max(np.abs(out - ref)) / np.max(np.abs(ref))
    print("fe err", err, "bucket", info["bucket"])
    assert err < 1e-13
    assert np.array_equal(out[:, loc < 0], pred[:, loc < 0])


def test_zero_volume_and_flipped_tetrahedra_and_empty_mesh():
    """Zero-volume tetrahedra are ignored, orientation does not matter, and a mesh with no
    tetrahedra leaves the predictor unchanged."""
    n = (8, 8, 8)
    lin = lambda x, y, z: x + 8 * (y + 8 * z)
    esp = np.array([lin(0, 0, 0), lin(6, 0, 0), lin(0, 6, 0), lin(0, 0, 6), lin(3, 3, 0)])
    tets = np.array([[0, 1, 2, 4], [1, 0, 2, 3]], np.int32)        # flat first, then flipped
    rng = np.random.default_rng(2)
    pred = rng.normal(size=(1, 512))
    vals = rng.normal(size=(1, 5))
    announce("fe: zero-volume and flipped tetrahedra")
    loc, out, info = _device_run(n, esp, tets, vals, pred)
    assert info["kept"] == 1
    xyz = _grid_xyz(n)
    assert np.array_equal(loc >= 0, xyz.sum(axis=1) <= 6) and set(np.unique(loc)) == {-1, 1}
    assert np.max(np.abs(out - O.fe_reconstruct(n, esp, tets, vals, pred))) < 1e-13
    announce("fe: empty mesh")
    loc, out, info = _device_run(n, esp, np.zeros((0, 4), np.int32), vals, pred)
    assert np.all(loc == -1) and np.array_equal(out, pred)


def test_bad_arguments_are_rejected():
    import torch
    from paper_1907_02604_amd import sgq
    n = (8, 8, 8)
    with pytest.raises(sgq.SgqError):
        sgq.FeMesh(n, [0, 7, 56, 448], [[0, 1, 2, 4]])             # vertex out of range
    with pytest.raises(sgq.SgqError):
        sgq.FeMesh(n, [0, 7, 56, 512], [[0, 1, 2, 3]])             # ESP outside the grid
    mesh = sgq.FeMesh(n, [0, 7, 56, 448], [[0, 1, 2, 3]], max_fields=1)
    v = torch.zeros(2, 4, dtype=torch.float64, device="cuda")
    p = torch.zeros(2, 512, dtype=torch.float64, device="cuda")
    with pytest.raises(sgq.SgqError):
        mesh.reconstruct(v, p, torch.empty_like(p))                # more fields than planned
    mesh.close()


def test_density_chain_on_sampled_points():
    """rho at the ESPs from rho_quadrature, then the fine-grid density: against the oracle's
    own ESP densities through its own reconstruction, on sampled points of the 64^3 grid, at
    the FP32 path's bar."""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2).subset(np.arange(40))
    esp = P.centers
    tets = synth.esp_mesh(P.n, esp)
    sites = synth.hcp_sites(P.L)
    pred = synth.predictor_fields(P.n, P.h, sites)[:1]
    plan = sgq.Plan.from_problem(P)
    v, R, E, _ = sgq.device_inputs(P)
    rho = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    announce("fe chain: density at 40 ESPs, reconstruction on 64^3")
    sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho)
    mesh = sgq.FeMesh(P.n, esp, tets, max_fields=1)
    p = torch.as_tensor(pred.reshape(1, -1), device="cuda")
    out = torch.empty_like(p)
    mesh.reconstruct(rho.reshape(1, -1), p, out)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    rho_ref, _ = O.rho_quadrature(P)
    loc = torch.empty(p.shape[1], dtype=torch.int32, device="cuda")
    mesh.location(loc)
    torch.cuda.synchronize()
    loc = loc.cpu().numpy()
    rng = np.random.default_rng(11)
    sample = np.concatenate([rng.choice(np.nonzero(loc >= 0)[0], 300, replace=False),
                             rng.choice(np.nonzero(loc < 0)[0], 50, replace=False), esp[:5]])
    ref = O.fe_reconstruct(P.n, esp, tets, rho_ref[None, :], pred, points=sample)
    got = out.cpu().numpy()[:, sample]
    err = O.normwise_rel_err(got.ravel(), ref.ravel())
    print("chain err", err)
    assert err < 1e-4
    assert np.max(np.abs(got[0, -5:] - rho.cpu().numpy()[:5])) <= 1e-12 * np.max(np.abs(got))
    mesh.close()
    plan.close()


def test_full_size_coarse_grained_128_grid():
    """The measured workload: 128^3 fine grid, ESPs = the full-resolution cylinder of radius
    4 around the core line plus 65536 seeded points, Delaunay mesh, two fields.  Location
    of sampled points against the oracle's brute force; every ESP reproduces its value;
    a linear corrector is reproduced at every located point; points outside keep the
    predictor bit for bit; sampled fields against the oracle."""
    import torch
    from paper_1907_02604_amd import sgq
    n = (128, 128, 128)
    esp = synth.coarse_esps(n, 5, 65536, 4)
    announce(f"fe full size: meshing {esp.size} ESPs")
    tets = synth.esp_mesh(n, esp)
    rng = np.random.default_rng(12)
    npts = int(np.prod(n))
    pred = rng.normal(size=(2, npts))
    X = O.esp_coords(n, esp).astype(np.float64)
    coef = np.array([[0.3, 1e-3, -2e-3, 5e-4], [-1.0, 2e-3, 1e-3, -1e-3]])
    vals = pred[:, esp] + coef[:, :1] + coef[:, 1:] @ X.T
    announce(f"fe full size: {len(tets)} tets, locate + reconstruct")
    loc, out, info = _device_run(n, esp, tets, vals, pred)
    print("mesh", info)
    xyz = _grid_xyz(n)
    inside = loc >= 0
    assert np.all(inside[esp])
    assert np.max(np.abs(out[:, esp] - vals)) <= 1e-12 * np.max(np.abs(vals))
    lin = pred[:, inside] + coef[:, :1] + coef[:, 1:] @ xyz[inside].T.astype(np.float64)
    assert np.max(np.abs(out[:, inside] - lin)) <= 1e-11
    assert np.array_equal(out[:, ~inside], pred[:, ~inside])
    sample = np.concatenate([rng.choice(npts, 120, replace=False),
                             rng.choice(np.nonzero(~inside)[0], 20, replace=False)])
    announce("fe full size: oracle location of 140 sampled points")
    assert np.array_equal(loc[sample], O.fe_locate(n, esp, tets, xyz[sample]))
    vals2 = rng.normal(size=(2, esp.size))
    _, out2, _ = _device_run(n, esp, tets, vals2, pred)
    ref = O.fe_reconstruct(n, esp, tets, vals2, pred, points=sample[:60])
    assert np.max(np.abs(out2[:, sample[:60]] - ref)) <= 1e-13 * np.max(np.abs(ref))
