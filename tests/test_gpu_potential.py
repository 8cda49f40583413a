"""Exchange-correlation, periodic Poisson and effective potential (sgq_lda_xc, sgq_poisson,
sgq_effective_potential) on the GPU against the FP64 oracle."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1907_02604_amd import synth
from gpu_util import announce, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def test_lda_xc_matches_oracle():
    import torch
    from paper_1907_02604_amd import sgq
    rng = np.random.default_rng(1)
    rho = np.concatenate([10.0 ** rng.uniform(-8, 1.7, size=100000), [0.0, -1e-3, 1e-300]])
    r = torch.as_tensor(rho, device="cuda")
    v = torch.empty_like(r)
    e = torch.empty_like(r)
    announce("lda xc: 100003 densities over ten decades")
    sgq.lda_xc(r, v, e)
    torch.cuda.synchronize()
    ref_e, ref_u = O.lda_xc(rho)
    ge, gu = e.cpu().numpy(), v.cpu().numpy()
    pos = rho > 1e-200
    assert np.max(np.abs(gu[pos] - ref_u[pos]) / np.abs(ref_u[pos])) < 1e-13
    assert np.max(np.abs(ge[pos] - ref_e[pos]) / np.abs(ref_e[pos])) < 1e-13
    assert np.all(gu[rho <= 0] == 0.0) and np.all(ge[rho <= 0] == 0.0)


@pytest.mark.parametrize("shape", [(12, 10, 8), (16, 16, 16), (9, 20, 30), (5, 6, 1), (1, 1, 1),
                                   (25, 24, 27), (64, 64, 64), (128, 96, 80), (8, 256, 256)])
def test_poisson_matches_oracle(shape):
    """phi against the oracle's FFT solve (every radix 4, 2, 3, 5 and degenerate axes), the
    reported mean, and the real-space stencil residual of the device result (the last shape:
    256-point x and y lines, the longest tiles of the line passes)."""
    import torch
    from paper_1907_02604_amd import sgq
    nz, ny, nx = shape
    rng = np.random.default_rng(sum(shape))
    s = rng.normal(size=shape) + 0.3
    h = 0.45
    pot = sgq.Potential((nx, ny, nz), h)
    sd = torch.as_tensor(s, device="cuda")
    phi = torch.empty_like(sd)
    mean = torch.empty(1, dtype=torch.float64, device="cuda")
    announce(f"poisson {shape}")
    pot.poisson(sd, phi, mean)
    torch.cuda.synchronize()
    ref, ref_mean = O.poisson_periodic(s, h)
    got = phi.cpu().numpy()
    scale = max(np.max(np.abs(ref)), 1e-300)
    print(shape, "err", np.max(np.abs(got - ref)) / scale)
    assert np.max(np.abs(got - ref)) <= 1e-12 * scale + 1e-15
    assert abs(mean.item() - ref_mean) < 1e-14
    lap = -2.0 * O.kinetic_apply(got, h, periodic=True)
    assert np.max(np.abs(-lap / (4 * math.pi) - (s - s.mean()))) < 1e-10 * np.max(np.abs(s))
    pot.close()


def test_effective_potential_matches_oracle():
    """V = phi[rho + b] + u(rho), phi, e_xc and the mean, on a C2-sized 64^3 grid with a
    positive synthetic density and the Gaussian nuclear charges of the C2 atoms."""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2)
    rho = synth.predictor_fields(P.n, P.h, P.atoms)[0] + 1e-4
    b = synth.nuclear_charge(P.n, P.h, P.atoms)
    pot = sgq.Potential(P.n, P.h)
    r = torch.as_tensor(rho, device="cuda")
    bd = torch.as_tensor(b, device="cuda")
    v, phi, exc = torch.empty_like(r), torch.empty_like(r), torch.empty_like(r)
    mean = torch.empty(1, dtype=torch.float64, device="cuda")
    announce("effective potential 64^3")
    pot.effective(r, v, b=bd, phi=phi, exc=exc, mean=mean)
    torch.cuda.synchronize()
    rV, rE, rP, rM = O.effective_potential(rho, b, P.h)
    for got, ref in ((v, rV), (phi, rP), (exc, rE)):
        g = got.cpu().numpy()
        assert np.max(np.abs(g - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert abs(mean.item() - rM) < 1e-14
    # without b and outputs beyond v
    v2 = torch.empty_like(r)
    pot.effective(r, v2)
    torch.cuda.synchronize()
    rV2, _, _, _ = O.effective_potential(rho, np.zeros_like(rho), P.h)
    assert np.max(np.abs(v2.cpu().numpy() - rV2)) <= 1e-12 * np.max(np.abs(rV2))
    pot.close()


def test_full_size_128_grid_and_repeatability():
    """The measured workload's grid (128^3): V against the oracle everywhere, bitwise equal
    on a second call."""
    import torch
    from paper_1907_02604_amd import sgq
    n = (128, 128, 128)
    sites = synth.hcp_sites((64.0, 64.0, 64.0))
    rho = synth.predictor_fields(n, 0.5, sites)[0] + 1e-4
    b = synth.nuclear_charge(n, 0.5, sites)
    pot = sgq.Potential(n, 0.5)
    r = torch.as_tensor(rho, device="cuda")
    bd = torch.as_tensor(b, device="cuda")
    v, v2 = torch.empty_like(r), torch.empty_like(r)
    announce("effective potential 128^3")
    pot.effective(r, v, b=bd)
    pot.effective(r, v2, b=bd)
    torch.cuda.synchronize()
    assert torch.equal(v, v2)
    rV, _, _, _ = O.effective_potential(rho, b, 0.5)
    assert np.max(np.abs(v.cpu().numpy() - rV)) <= 1e-12 * np.max(np.abs(rV))
    pot.close()


def test_bad_grids_are_rejected():
    from paper_1907_02604_amd import sgq
    for n, h in (((7, 8, 8), 0.5), ((8, 8, 8), 0.0), ((4096, 1, 1), 0.5), ((0, 4, 4), 0.5)):
        with pytest.raises(sgq.SgqError):
            sgq.Potential(n, h)
