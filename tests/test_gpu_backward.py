"""GPU parity of band_energy_backward (the hand-written adjoint) against the FP64 oracle
gradient and central finite differences."""
import numpy as np
import pytest

import oracle as O
from oracle_util import custom_problem, lin, smooth_random_potential
from paper_1907_02604_amd import synth
from gpu_util import announce, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def _small_system(seed=0, K=7):
    N, h = 16, 0.5
    rng = np.random.default_rng(seed)
    atoms = rng.uniform(0, N * h, size=(5, 3))
    E = rng.uniform(-1, 1, size=(5, 4))
    P = custom_problem(N, h=h, atoms=atoms, proj_E=E, v_loc=synth.gaussian_vloc((N,) * 3, h, atoms),
                       centers=np.zeros(4, np.int64), half_width=4, depth=K, mu=-0.5, kT=0.3)
    P.weight[:] = rng.uniform(0.5, 2.0, size=4)
    for i in range(4):
        g = np.floor(atoms[i] / h).astype(int) % N
        P.centers[i] = lin(g[0], g[1], g[2], N)
    return P


def _gpu_grad(P, kind, precision, grad_omega=1.0):
    import torch
    from paper_1907_02604_amd import sgq
    prec = sgq.SGQ_FP64 if precision == "f64" else sgq.SGQ_FP32
    plan = sgq.Plan(P.n, P.h, P.atoms.shape[0], P.n_proj, P.centers, P.half_width, P.depth, prec)
    dV, dR, dE = sgq.energy_backward(P, kind, grad_omega, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == 0
    out = dV.cpu().numpy(), dR.cpu().numpy(), dE.cpu().numpy()
    plan.close()
    return out


def _rel(a, b):
    return O.normwise_rel_err(a, b)


@pytest.mark.parametrize("kind", [O.FREE, O.BAND, O.GRAND])
def test_small_system_matches_oracle_gradient(kind):
    P = _small_system()
    rdV, rdE, rdR = O.band_energy_backward(P, kind=kind, grad_omega=1.3)
    announce(f"bwd small fp64 kind={kind}")
    dV, dR, dE = _gpu_grad(P, kind, "f64", 1.3)
    assert _rel(dV, rdV) < 1e-6
    assert _rel(dR, rdR) < 1e-6
    assert _rel(dE, rdE) < 1e-6
    announce(f"bwd small fp32 kind={kind}")
    dV, dR, dE = _gpu_grad(P, kind, "f32", 1.3)
    print("fp32 grad errs", _rel(dV, rdV), _rel(dR, rdR), _rel(dE, rdE))
    assert _rel(dV, rdV) < 1e-4
    assert _rel(dR, rdR) < 1e-4
    assert _rel(dE, rdE) < 1e-4


def test_gpu_gradient_matches_gpu_central_differences():
    """FP64 path: the adjoint against central differences of the GPU forward (step 1e-4)."""
    import torch
    from paper_1907_02604_amd import sgq
    P = _small_system(seed=3)
    announce("bwd vs fd fp64")
    dV, dR, dE = _gpu_grad(P, O.FREE, "f64")
    plan = sgq.Plan(P.n, P.h, P.atoms.shape[0], P.n_proj, P.centers, P.half_width, P.depth, sgq.SGQ_FP64)
    v, R, E, w = sgq.device_inputs(P)
    e = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")

    def omega(vv=None, RR=None, EE=None):
        sgq.band_energy(plan, v if vv is None else vv, R if RR is None else RR,
                        E if EE is None else EE, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
        return float(om.item())

    step = 1e-4
    H0 = O.NodeHamiltonian(P, 0)
    rng = np.random.default_rng(0)
    for _ in range(3):
        iz, iy, ix = rng.choice(H0.gz), rng.choice(H0.gy), rng.choice(H0.gx)
        vp, vm = v.clone(), v.clone()
        vp[iz, iy, ix] += step
        vm[iz, iy, ix] -= step
        fd = (omega(vv=vp) - omega(vv=vm)) / (2 * step)
        assert dV[iz, iy, ix] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    for J, l in [(0, 1), (2, 3)]:
        Ep, Em = E.clone(), E.clone()
        Ep[J, l] += step
        Em[J, l] -= step
        fd = (omega(EE=Ep) - omega(EE=Em)) / (2 * step)
        assert dE[J, l] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    # positions: projectors move with the atom, V_loc held fixed (the nonlocal part)
    for J, a in [(0, 0), (1, 2)]:
        Rp, Rm = R.clone(), R.clone()
        Rp[J, a] += step
        Rm[J, a] -= step
        fd = (omega(RR=Rp) - omega(RR=Rm)) / (2 * step)
        assert dR[J, a] == pytest.approx(fd, rel=2e-6, abs=1e-8)
    plan.close()


def test_local_potential_chain_rule():
    """dOmega/dR including V_loc(R): library chain-rule kernel vs the oracle's."""
    import torch
    from paper_1907_02604_amd import sgq
    P = _small_system(seed=5)
    rdV, _, rdR = O.band_energy_backward(P, kind=O.FREE)
    ref = rdR + O.vloc_position_gradient(rdV, P.n, P.h, P.atoms, synth.VLOC_DEPTH, synth.VLOC_SIGMA,
                                         synth.VLOC_CUTOFF_SIGMAS)
    plan = sgq.Plan(P.n, P.h, P.atoms.shape[0], P.n_proj, P.centers, P.half_width, P.depth, sgq.SGQ_FP64)
    announce("vloc chain rule")
    dV, dR, dE = sgq.energy_backward(P, sgq.SGQ_FREE, plan=plan)
    R = torch.as_tensor(P.atoms, dtype=torch.float64, device="cuda")
    sgq.vloc_gaussian_backward(plan, dV, R, synth.VLOC_DEPTH, synth.VLOC_SIGMA,
                               synth.VLOC_CUTOFF_SIGMAS, dR)
    torch.cuda.synchronize()
    assert _rel(dR.cpu().numpy(), ref) < 1e-6
    plan.close()


def test_autograd_function():
    import torch
    from paper_1907_02604_amd import sgq
    P = _small_system(seed=7)
    plan = sgq.Plan(P.n, P.h, P.atoms.shape[0], P.n_proj, P.centers, P.half_width, P.depth, sgq.SGQ_FP64)
    v, R, E, w = sgq.device_inputs(P)
    v.requires_grad_(True)
    R.requires_grad_(True)
    E.requires_grad_(True)
    announce("autograd")
    om = sgq.band_energy_fn(v, R, E, plan, w, P.mu, P.kT, sgq.SGQ_FREE,
                            vloc_model=(synth.VLOC_DEPTH, synth.VLOC_SIGMA, synth.VLOC_CUTOFF_SIGMAS))
    (2.0 * om).backward()
    rdV, rdE, rdR = O.band_energy_backward(P, kind=O.FREE, grad_omega=2.0)
    rdR = rdR + O.vloc_position_gradient(rdV, P.n, P.h, P.atoms, synth.VLOC_DEPTH, synth.VLOC_SIGMA,
                                         synth.VLOC_CUTOFF_SIGMAS)
    assert _rel(v.grad.cpu().numpy(), rdV) < 1e-6
    assert _rel(E.grad.cpu().numpy(), rdE) < 1e-6
    assert _rel(R.grad.cpu().numpy(), rdR) < 1e-6
    assert om.item() == pytest.approx(O.band_energy(P, kind=O.FREE)[1], rel=1e-9)
    plan.close()


def test_hellmann_feynman_on_gpu():
    """GRAND, untruncated, every node, K = dim: dOmega/dV = rho h^3 (FP64 path)."""
    import torch
    from paper_1907_02604_amd import sgq
    N, h = 3, 0.5
    P = custom_problem(N, h=h, v_loc=smooth_random_potential(N, 9), depth=27, mu=1.0, kT=0.4)
    plan = sgq.Plan(P.n, P.h, 0, 0, P.centers, P.half_width, P.depth, sgq.SGQ_FP64)
    announce("HF identity")
    dV, _, _ = sgq.energy_backward(P, sgq.SGQ_GRAND, plan=plan)
    rho, _ = sgq.rho(P, plan=plan)
    torch.cuda.synchronize()
    np.testing.assert_allclose(dV.cpu().numpy().ravel(), rho.cpu().numpy() * h ** 3, rtol=1e-9, atol=1e-13)
    plan.close()


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-6)])
@pytest.mark.parametrize("seed", [21, 22, 23, 24])
def test_differentiation_workload_subset(precision, tol, seed):
    """48^3 grid, 16 atoms, 33^3 cubes, K = 60 (the differentiation workload) on a node
    subset: dV, dR (nonlocal) and dE against the oracle gradient, every output within the
    precision's bar.  Seed 21's subset holds a node with a Gauss point 2.7 kT above mu, the
    case most sensitive to the rounding of the FP32 matvec."""
    P = synth.make_problem(4)
    idx = np.random.default_rng(seed).choice(P.n_nodes, 6, replace=False)
    Q = P.subset(idx)
    rdV, rdE, rdR = O.band_energy_backward(Q, kind=O.FREE)
    announce(f"C4 subset bwd {precision} seed {seed}")
    dV, dR, dE = _gpu_grad(Q, O.FREE, precision)
    print("C4 grad errs", _rel(dV, rdV), _rel(dR, rdR), _rel(dE, rdE))
    assert _rel(dV, rdV) < tol
    assert _rel(dR, rdR) < tol
    assert _rel(dE, rdE) < tol


def test_dislocation_workload_subset():
    """128^3 screw-displaced lattice, cubes 25^3..49^3, K = 80, node weights 32: FP32, every
    adjoint output within 1e-4 of the oracle gradient."""
    P = synth.make_problem(5)
    from gpu_util import stratified_sample
    Q = P.subset(stratified_sample(P, 2, seed=22))
    rdV, rdE, rdR = O.band_energy_backward(Q, kind=O.FREE)
    announce("C5 subset bwd fp32")
    dV, dR, dE = _gpu_grad(Q, O.FREE, "f32")
    print("C5 grad errs", _rel(dV, rdV), _rel(dR, rdR), _rel(dE, rdE))
    assert _rel(dV, rdV) < 1e-4
    assert _rel(dR, rdR) < 1e-4
    assert _rel(dE, rdE) < 1e-4


def test_backward_bitwise_deterministic():
    P = synth.make_problem(4).subset(np.arange(40))
    announce("bwd determinism")
    a = _gpu_grad(P, O.FREE, "f32")
    b = _gpu_grad(P, O.FREE, "f32")
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_nodes_beyond_every_projector(precision):
    """13^3 cubes of the differentiation workload that no projector reaches, in a plan with
    projectors (mu and kT raised so that the cubes hold charge): density and dV match the
    oracle, whose nonlocal sum is empty there, and the projector adjoints are exactly 0."""
    import dataclasses
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(4)
    Q = P.subset(np.arange(0, P.n_nodes, 211))
    Q.half_width[:] = 6
    far = []
    for q in range(Q.n_nodes):
        if O.NodeHamiltonian(Q, q).chi is None:
            far.append(q)
            if len(far) == 3:
                break
    Q = dataclasses.replace(Q.subset(far), precision=precision, mu=0.5, kT=0.2)
    Q.depth[:] = 12
    announce(f"nodes beyond every projector, {precision}")
    rho, _ = sgq.rho(Q)
    dV, dR, dE = sgq.energy_backward(Q, sgq.SGQ_FREE, 1.0)
    torch.cuda.synchronize()
    tol = 1e-6 if precision == "f64" else 1e-4
    ref_rho, _ = O.rho_quadrature(Q)
    rdV, rdE, rdR = O.band_energy_backward(Q, kind=O.FREE)
    assert not np.any(rdE) and not np.any(rdR)
    assert _rel(rho.cpu().numpy(), ref_rho) < tol
    assert _rel(dV.cpu().numpy(), rdV) < tol
    assert not torch.any(dR) and not torch.any(dE)


def test_deep_adjoint_on_the_uneven_workload():
    """96^3 uneven-batching workload: three stratified nodes (cubes 25^3..49^3) at depth
    100, past the former 80 cap of the adjoint; kT = 0.005.  FP64 within 1e-6 and FP32
    within 1e-4 of the oracle gradient, every output."""
    from gpu_util import stratified_sample
    P = synth.make_problem(3)
    Q = P.subset(stratified_sample(P, 3, seed=31))
    Q.depth[:] = 100
    rdV, rdE, rdR = O.band_energy_backward(Q, kind=O.FREE)
    for precision, tol in (("f64", 1e-6), ("f32", 1e-4)):
        announce(f"C3 deep adjoint {precision}")
        dV, dR, dE = _gpu_grad(Q, O.FREE, precision)
        errs = _rel(dV, rdV), _rel(dR, rdR), _rel(dE, rdE)
        print("C3 K=100 grad errs", precision, errs)
        assert max(errs) < tol


def test_wide_planes_take_the_512_lane_launch(monkeypatch):
    """The backward reverses FP32 cubes wider than 35 points (up to 49) in a 512-lane launch
    of their own, whose march takes planes that wide, and the other nodes in a 256-lane one.
    Three stratified nodes of the 128^3 screw lattice (cubes 25^3, 41^3 and 49^3, K = 80):
    the adjoint is within 1e-4 of the oracle gradient on every output, and the same bits
    whatever lanes per node the plan's forward uses.  After a 512-lane forward that retained
    the rows of the two wide nodes, their adjoint equals the recompute bit for bit, since
    the forward and the recompute run the same 512-lane sweeps."""
    import torch
    from paper_1907_02604_amd import sgq
    from gpu_util import stratified_sample
    P = synth.make_problem(5)
    Q = P.subset(stratified_sample(P, 3, seed=42))
    side = 2 * Q.half_width + 1
    assert sorted(side) == [25, 41, 49]
    rdV, rdE, rdR = O.band_energy_backward(Q, kind=O.FREE)

    def plan_512(prob):
        monkeypatch.setenv("SGQ_BLOCK", "512")
        monkeypatch.setenv("SGQ_WG_PER_CU", "1")
        plan = sgq.Plan.from_problem(prob)
        monkeypatch.delenv("SGQ_BLOCK")
        monkeypatch.delenv("SGQ_WG_PER_CU")
        return plan

    announce("C5 wide planes: adjoint, 256-lane plan")
    plan = sgq.Plan.from_problem(Q)
    rec = _gpu_grad_on(plan, Q)
    plan.close()
    print("C5 wide-plane grad errs", _rel(rec[0], rdV), _rel(rec[1], rdR), _rel(rec[2], rdE))
    for got, ref in zip(rec, (rdV, rdR, rdE)):
        assert _rel(got, ref) < 1e-4
    announce("C5 wide planes: adjoint, 512-lane plan")
    plan = plan_512(Q)
    rec512 = _gpu_grad_on(plan, Q)
    plan.close()
    for a, b, name in zip(rec512, rec, ("dV", "dR", "dE")):
        assert np.array_equal(a, b), name
    W = Q.subset(np.nonzero(side > 35)[0])
    plan = plan_512(W)
    announce("C5 wide planes: two wide nodes, recompute")
    wrec = _gpu_grad_on(plan, W)
    plan.set_retain(True)
    v, R, E, w = sgq.device_inputs(W)
    e = torch.empty(W.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    announce("C5 wide planes: 512-lane forward, retained adjoint")
    sgq.band_energy(plan, v, R, E, w, W.mu, W.kT, sgq.SGQ_FREE, e, om)
    wret = _gpu_grad_on(plan, W, (v, R, E, w))
    plan.close()
    for a, b, name in zip(wret, wrec, ("dV", "dR", "dE")):
        assert np.array_equal(a, b), name


@pytest.mark.parametrize("case", ["cube51", "periodic"])
def test_fp32_nodes_off_the_plane_march(case):
    """FP32 nodes that no plane march takes, reversed with separate dot, update and operator
    passes in the 256-lane launch: two 51^3 cubes (wider than the 512-lane march's 49-point
    planes) on a 60^3 grid with 24 projector atoms, or two untruncated nodes of a 16^3
    periodic grid with 4.  Every adjoint output within 1e-4 of the oracle gradient."""
    import dataclasses
    rng = np.random.default_rng(3)
    N, h = (60, 0.5) if case == "cube51" else (16, 0.5)
    na = 24 if case == "cube51" else 4
    atoms = rng.uniform(0, N * h, size=(na, 3))
    E = rng.uniform(-1, 1, size=(na, 4))
    centers = ([lin(30, 30, 30, N), lin(5, 50, 12, N)] if case == "cube51"
               else [lin(3, 4, 5, N), lin(10, 2, 7, N)])
    P = custom_problem(N, h=h, atoms=atoms, proj_E=E, v_loc=synth.gaussian_vloc((N,) * 3, h, atoms),
                       centers=centers, half_width=25 if case == "cube51" else -1,
                       depth=16 if case == "cube51" else 14, mu=-0.3, kT=0.05)
    P = dataclasses.replace(P, precision="f32")
    rdV, rdE, rdR = O.band_energy_backward(P, kind=O.FREE)
    announce(f"fp32 off the march: {case}")
    dV, dR, dE = _gpu_grad(P, O.FREE, "f32")
    errs = _rel(dV, rdV), _rel(dR, rdR), _rel(dE, rdE)
    print("off-march grad errs", case, errs)
    assert max(errs) < 1e-4


def _gpu_grad_on(plan, P, inputs=None):
    """(dV, dR, dE) on host through an existing plan, on the given device inputs (the ones a
    forward saw, for its retained rows) or fresh copies."""
    import torch
    from paper_1907_02604_amd import sgq
    v, R, E, w = inputs or sgq.device_inputs(P)
    plan.prepare_backward()
    g = torch.ones(1, dtype=torch.float64, device="cuda")
    dV = torch.empty_like(v)
    dR = torch.zeros_like(R)
    dE = torch.zeros_like(E)
    sgq.band_energy_backward(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, g, dV, dR, dE)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    return dV.cpu().numpy(), dR.cpu().numpy(), dE.cpu().numpy()


def test_every_reverse_path_in_one_plan():
    """One FP32 plan on a 60^3 grid with 24 projector atoms whose five nodes take every
    reverse path of the backward: cubes of 25^3 and 33^3 (the 256-lane plane march), 41^3
    (the 512-lane launch), 51^3 (wider than either march: separate dot, update and operator
    passes) and an untruncated node of the periodic grid.  The split node queue serves both
    launches in one call; every adjoint output is within 1e-4 of the oracle gradient, without
    and with a forward first (whose stored tridiagonals the eigensolve pre-pass then takes)."""
    import dataclasses
    import torch
    from paper_1907_02604_amd import sgq
    N, h = 60, 0.5
    rng = np.random.default_rng(5)
    atoms = rng.uniform(0, N * h, size=(24, 3))
    E = rng.uniform(-1, 1, size=(24, 4))
    centers = [lin(30, 30, 30, N), lin(5, 50, 12, N), lin(44, 9, 27, N), lin(17, 38, 51, N),
               lin(2, 3, 4, N)]
    P = custom_problem(N, h=h, atoms=atoms, proj_E=E, v_loc=synth.gaussian_vloc((N,) * 3, h, atoms),
                       centers=centers, half_width=12, depth=16, mu=-0.3, kT=0.05)
    P.half_width[:] = [12, 20, 25, 16, -1]
    P = dataclasses.replace(P, precision="f32")
    rdV, rdE, rdR = O.band_energy_backward(P, kind=O.FREE)
    announce("every reverse path: backward alone")
    plan = sgq.Plan.from_problem(P)
    got = _gpu_grad_on(plan, P)
    plan.close()
    errs = _rel(got[0], rdV), _rel(got[1], rdR), _rel(got[2], rdE)
    print("mixed-path grad errs", errs)
    assert max(errs) < 1e-4
    announce("every reverse path: forward, then backward")
    plan = sgq.Plan.from_problem(P)
    plan.prepare_backward()
    v, R, Ed, w = sgq.device_inputs(P)
    e = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    sgq.band_energy(plan, v, R, Ed, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
    fwd = _gpu_grad_on(plan, P, (v, R, Ed, w))
    plan.close()
    errs = _rel(fwd[0], rdV), _rel(fwd[1], rdR), _rel(fwd[2], rdE)
    print("mixed-path grad errs after a forward", errs)
    assert max(errs) < 1e-4


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-6)])
def test_chained_projector_boxes(precision, tol):
    """Projector atoms whose boxes overlap in long chains, so the scatter of the atoms
    outside the parallel group runs in many layers: 24 atoms one grid point apart on a line
    (each box overlaps the six before it, one layer per atom) and a 3 x 3 x 3 cluster 1.5
    grid points apart (27 boxes that all overlap), both inside the cubes of two nodes on a
    32^3 grid.  Density, rule depth and every adjoint output against the oracle."""
    import dataclasses
    from gpu_util import gpu_rho
    N, h = 32, 0.5
    rng = np.random.default_rng(9)
    line = [[(4 + i) * h + 0.1, 16 * h + 0.13, 16 * h - 0.07] for i in range(24)]
    cluster = [[(8 + 1.5 * a) * h + 0.05, (8 + 1.5 * b) * h, (24 + 1.5 * c) * h - 0.1]
               for a in range(3) for b in range(3) for c in range(3)]
    atoms = np.array(line + cluster)
    E = rng.uniform(-0.5, 0.5, size=(atoms.shape[0], 4))
    P = custom_problem(N, h=h, atoms=atoms, proj_E=E, v_loc=smooth_random_potential(N, 5, 0.3),
                       centers=[lin(16, 16, 16, N), lin(10, 10, 22, N)], half_width=8,
                       depth=16, mu=0.0, kT=0.1)
    P = dataclasses.replace(P, precision=precision)
    ref_rho, ref_k = O.rho_quadrature(P)
    rdV, rdE, rdR = O.band_energy_backward(P, kind=O.FREE)
    announce(f"chained projector boxes {precision}: density")
    rho, ke, status = gpu_rho(P)
    assert status == 0
    assert np.array_equal(ke, ref_k)
    assert O.normwise_rel_err(rho, ref_rho) < tol
    announce(f"chained projector boxes {precision}: adjoint")
    dV, dR, dE = _gpu_grad(P, O.FREE, precision)
    errs = _rel(dV, rdV), _rel(dR, rdR), _rel(dE, rdE)
    print("chained-box errs", precision, errs)
    assert max(errs) < tol


@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("f64", 1e-6)])
def test_projector_boxes_over_one_round(precision, tol):
    """A grid spacing of 0.4 bohr makes the projector box 9^3 = 729 points, more than the
    6 x 64 box points one round of the adjoint's box sums covers, so the sums take the path
    that goes over each atom's box in several rounds.  Two 13^3 nodes centred on atoms of
    a 24^3 grid with 10 projector atoms: density, rule depth and every adjoint output
    against the oracle."""
    import dataclasses
    from gpu_util import gpu_rho
    N, h = 24, 0.4
    rng = np.random.default_rng(4)
    atoms = rng.uniform(0, N * h, size=(10, 3))
    E = rng.uniform(-0.6, 0.6, size=(10, 4))
    g = np.rint(atoms[:2] / h).astype(int) % N
    P = custom_problem(N, h=h, atoms=atoms, proj_E=E, v_loc=smooth_random_potential(N, 7, 0.3),
                       centers=[lin(*g[0], N), lin(*g[1], N)], half_width=6, depth=12,
                       mu=0.3, kT=0.1)
    P = dataclasses.replace(P, precision=precision)
    ref_rho, ref_k = O.rho_quadrature(P)
    rdV, rdE, rdR = O.band_energy_backward(P, kind=O.FREE)
    announce(f"projector boxes of 9^3 {precision}: density")
    rho, ke, status = gpu_rho(P)
    assert status == 0
    assert np.array_equal(ke, ref_k)
    assert O.normwise_rel_err(rho, ref_rho) < tol
    announce(f"projector boxes of 9^3 {precision}: adjoint")
    dV, dR, dE = _gpu_grad(P, O.FREE, precision)
    errs = _rel(dV, rdV), _rel(dR, rdR), _rel(dE, rdE)
    print("9^3-box errs", precision, errs)
    assert max(errs) < tol
