"""GPU parity of rho_quadrature / band_energy against the FP64 oracle (MI355X)."""
import numpy as np
import pytest

import oracle as O
from oracle_util import (custom_problem, lin, oracle_rho_pool, per_node_rel_err,
                         smooth_random_potential)
from paper_1907_02604_amd import synth
from gpu_util import (announce, gpu_energy, gpu_rho, gpu_rho_bench_launch, needs_gpu, oracle_rho,
                      stratified_sample)

pytestmark = [pytest.mark.gpu, needs_gpu]

FP64_TOL = 1e-6     # normwise relative, FP64 path
FP32_TOL = 1e-4     # normwise relative, FP32 matvecs with FP64 dots / tridiagonal / quadrature


def test_c1_periodic_fp64_all_nodes():
    """16^3 periodic, K = 30, FP64, all 4096 nodes on the GPU; oracle on a sample."""
    P = synth.make_problem(1)
    announce("C1 fp64 4096 nodes")
    rho, keff, st = gpu_rho(P)
    assert st == 0
    assert np.all(keff == 30)
    sample = np.random.default_rng(11).choice(P.n_nodes, 160, replace=False)
    ref, _ = oracle_rho(P, sample)
    err = O.normwise_rel_err(rho[sample], ref)
    print("C1 normwise err", err)
    assert err < FP64_TOL
    assert np.all(np.isfinite(rho)) and rho.min() > 0


def test_c2_fp32_and_fp64_paths():
    """64^3, 33^3 cubes, K = 60, projectors: FP32 path within 1e-4 and FP64 within 1e-6."""
    P = synth.make_problem(2).subset(np.arange(24))
    ref, _ = oracle_rho(P, range(P.n_nodes))
    announce("C2 fp32 24 nodes")
    r32, k32, st = gpu_rho(P)
    assert st == 0 and np.all(k32 == 60)
    announce("C2 fp64 24 nodes")
    r64, k64, st = gpu_rho(P, precision="f64")
    assert st == 0
    e32 = O.normwise_rel_err(r32, ref)
    e64 = O.normwise_rel_err(r64, ref)
    print("C2 normwise err fp32 %.3e fp64 %.3e" % (e32, e64))
    assert e32 < FP32_TOL
    assert e64 < FP64_TOL


def test_c2_full_launch_sampled():
    """The full 8192-node workload in the benchmark's launch configuration (autotuned,
    graph-replayed on a side stream); 256 sampled nodes against the oracle, normwise and per
    node (nodes above 1e-3 of the largest density, where the normwise bar implies at most
    0.1)."""
    P = synth.make_problem(2)
    announce("C2 fp32 8192 nodes, benchmark launch")
    rho, keff, st, shape = gpu_rho_bench_launch(P)
    print("C2 launch shape", shape)
    assert st == 0 and np.all(keff == 60)
    sample = np.random.default_rng(12).choice(P.n_nodes, 256, replace=False)
    ref = oracle_rho_pool(P, sample)
    err = O.normwise_rel_err(rho[sample], ref)
    pn = per_node_rel_err(rho[sample], ref)
    print("C2 full sampled err", err, "per node", pn)
    assert err < FP32_TOL
    assert pn < FP32_TOL / 1e-3


def test_c3_uneven_full_launch_sampled():
    """96^3, 20000 nodes with cube sides 25..49 and depths 40..100 in one launch, in the
    benchmark's launch configuration (autotuned, graph-replayed on a side stream)."""
    P = synth.make_problem(3)
    announce("C3 fp32 20000 nodes, benchmark launch")
    rho, keff, st, shape = gpu_rho_bench_launch(P)
    print("C3 launch shape", shape)
    assert st == 0
    assert np.array_equal(keff, P.depth)
    sample = stratified_sample(P, 96, seed=13)
    ref = oracle_rho_pool(P, sample)
    err = O.normwise_rel_err(rho[sample], ref)
    pn = per_node_rel_err(rho[sample], ref)
    print("C3 sampled err", err, "per node", pn)
    assert err < FP32_TOL
    assert pn < FP32_TOL / 1e-3


def test_c5_screw_subset():
    P = synth.make_problem(5)
    sample = stratified_sample(P, 4, seed=14)
    Q = P.subset(sample)
    announce("C5 fp32 4 nodes")
    rho, keff, st = gpu_rho(Q)
    assert st == 0
    ref, _ = oracle_rho(Q, range(Q.n_nodes))
    err = O.normwise_rel_err(rho, ref)
    print("C5 err", err)
    assert err < FP32_TOL


@pytest.mark.parametrize("kind", [O.FREE, O.BAND, O.GRAND])
def test_c4_band_energy(kind):
    P = synth.make_problem(4)
    idx = np.random.default_rng(15).choice(P.n_nodes, 10, replace=False)
    Q = P.subset(idx)
    Q.weight[:] = np.linspace(0.5, 2.0, Q.n_nodes)
    ref_e, ref_om = O.band_energy(Q, kind=kind)
    announce(f"C4 band_energy kind={kind}")
    e, om = gpu_energy(Q, kind)
    err = O.normwise_rel_err(e, ref_e)
    print("C4 e err", err, "omega", om, ref_om)
    assert err < FP32_TOL
    assert abs(om - ref_om) <= FP32_TOL * np.sum(np.abs(Q.weight * ref_e))
    e64, om64 = gpu_energy(Q, kind, precision="f64")
    assert O.normwise_rel_err(e64, ref_e) < FP64_TOL
    assert abs(om64 - ref_om) <= FP64_TOL * np.sum(np.abs(Q.weight * ref_e))


def test_rule_output_matches_oracle():
    """(theta_k, w_k) of each node and K_eff, FP64 path."""
    P = synth.make_problem(2, grid=32, n_nodes=6)
    P.half_width[:] = 10
    P.depth[:] = np.array([1, 2, 5, 17, 30, 40])
    announce("rule output fp64")
    rho, keff, st, tw = gpu_rho(P, want_rule=True, precision="f64")
    assert st == 0
    for q in range(P.n_nodes):
        th, w, k = O.node_rule(P, q)
        assert keff[q] == k
        np.testing.assert_allclose(tw[q, :k, 0], th, rtol=1e-9, atol=1e-9)
        np.testing.assert_allclose(tw[q, :k, 1], w, atol=1e-9)
        assert np.all(tw[q, k:] == 0)


def test_depth_one_is_fermi_of_diagonal():
    P = synth.make_problem(2, grid=32, n_nodes=5)
    P.half_width[:] = 8
    P.depth[:] = 1
    announce("K=1")
    rho, keff, st = gpu_rho(P, precision="f64")
    for q in range(P.n_nodes):
        H = O.NodeHamiltonian(P, q)
        e = H.start_vector()
        hcc = e @ H.apply(e)
        assert rho[q] == pytest.approx(2 / P.h ** 3 * O.fermi(np.array([hcc]), P.mu, P.kT)[0], rel=1e-12)


def test_nodes_at_grid_corners_and_seams():
    """Cubes that wrap through the periodic faces, with projector atoms near the seam."""
    N = 40
    P = synth.make_problem(2, grid=N, n_nodes=4)
    P.centers = np.array([0, N ** 3 - 1, lin(N - 1, 0, N // 2, N), lin(2, N - 3, 1, N)], dtype=np.int64)
    P.half_width[:] = np.array([16, 12, 9, 5])
    P.depth[:] = 25
    ref, _ = oracle_rho(P, range(4))
    announce("corner nodes fp32/fp64")
    r32, _, st = gpu_rho(P)
    assert st == 0
    r64, _, _ = gpu_rho(P, precision="f64")
    assert O.normwise_rel_err(r32, ref) < FP32_TOL
    assert O.normwise_rel_err(r64, ref) < FP64_TOL


def test_tiny_periodic_grid_breakdown_and_aliasing():
    """5^3 periodic grid (projector box wider than the grid, so images alias) and
    K > dim: Lanczos breaks down with K_eff <= 125 and the rule is exact."""
    N = 5
    P = custom_problem(N, h=0.5, atoms=[[0.6, 1.1, 2.2]], proj_E=[[0.4, -0.3, 0.2, 0.5]],
                       v_loc=smooth_random_potential(N, 4), centers=[0, 62, 124], depth=128,
                       mu=1.0, kT=0.5)
    ref, kref = oracle_rho(P, range(3))
    announce("tiny periodic fp64")
    rho, keff, st = gpu_rho(P, precision="f64")
    assert st == 0
    assert np.all(keff <= 125) and np.all(keff < 128)
    assert O.normwise_rel_err(rho, ref) < FP64_TOL


def test_empty_node_list():
    P = synth.make_problem(2, grid=32, n_nodes=1).subset([])
    announce("empty node list")
    rho, keff, st = gpu_rho(P)
    assert rho.size == 0 and st == 0


def test_nonfinite_potential_is_reported():
    from paper_1907_02604_amd import sgq
    import torch
    P = synth.make_problem(2, grid=32, n_nodes=3)
    P.half_width[:] = 6
    P.depth[:] = 10
    plan = sgq.Plan.from_problem(P)
    v, R, E, _ = sgq.device_inputs(P)
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    v[3, 4, 5] = float("nan")
    announce("non-finite potential")
    sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, out)
    assert plan.status() == sgq.SGQ_ENONFINITE
    v[3, 4, 5] = 0.0
    sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, out)
    assert plan.status() == sgq.SGQ_OK
    with pytest.raises(sgq.SgqError):
        sgq.rho_quadrature(plan, v, R, E, P.mu, -1.0, out)
    plan.close()


def test_bitwise_deterministic():
    P = synth.make_problem(2).subset(np.arange(64))
    announce("determinism")
    a, _, _ = gpu_rho(P)
    b, _, _ = gpu_rho(P)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("precision,tol", [("f32", FP32_TOL), ("f64", FP64_TOL)])
def test_plain_schedule_matches_oracle(precision, tol):
    """The per-node baseline schedule computes the same densities (64^3 workload, 6 nodes)."""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2).subset(np.arange(6))
    ref, _ = oracle_rho(P, range(P.n_nodes))
    prec = sgq.SGQ_FP64 if precision == "f64" else sgq.SGQ_FP32
    plan = sgq.Plan(P.n, P.h, P.atoms.shape[0], P.n_proj, P.centers, P.half_width, P.depth, prec)
    plan.set_schedule(sgq.SGQ_SCHEDULE_PLAIN)
    v, R, E, _ = sgq.device_inputs(P)
    rho = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    announce(f"plain schedule {precision}")
    sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho)
    torch.cuda.synchronize()
    assert plan.status() == 0
    err = O.normwise_rel_err(rho.cpu().numpy(), ref)
    print("plain err", err)
    assert err < tol
    plan.close()


def test_node_over_the_atom_limit_is_reported_and_skipped():
    """A node whose cube meets more atoms than the node state holds (300 atoms packed into a
    4-bohr box) latches SGQ_ELIMIT and gets NaN density, energy and Gauss rule, and its
    adjoint adds nothing; a node beyond the cluster is computed as usual and matches the
    oracle.  A Fermi-level solve on those rules reports the NaN rule, although it starts
    from a clear status word."""
    import torch
    from paper_1907_02604_amd import sgq
    N, h = 48, 0.5
    rng = np.random.default_rng(11)
    atoms = rng.uniform(2.0, 6.0, size=(300, 3))
    E = rng.uniform(-1.0, 1.0, size=(300, 4))
    centers = [lin(8, 8, 8, N), lin(32, 32, 32, N)]   # inside the cluster; 14 bohr away
    P = custom_problem(N, h=h, atoms=atoms, proj_E=E, v_loc=smooth_random_potential(N, 3, 0.3),
                       centers=centers, half_width=4, depth=12, mu=0.2, kT=0.1)
    plan = sgq.Plan.from_problem(P)
    announce("node over the atom limit: forward")
    rho, tw, _ = sgq.rho(P, plan=plan, want_rule=True)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_ELIMIT
    rho = rho.cpu().numpy()
    assert np.isnan(rho[0])
    rule = tw.cpu().numpy()
    assert np.all(np.isnan(rule[0])) and np.all(np.isfinite(rule[1]))
    far = P.subset([1])
    ref_rho, _ = O.rho_quadrature(far)
    assert abs(rho[1] - ref_rho[0]) < 1e-6 * abs(ref_rho[0])
    announce("node over the atom limit: Fermi level of its rules")
    res = torch.zeros(3, dtype=torch.float64, device="cuda")
    w = torch.ones(P.n_nodes, dtype=torch.float64, device="cuda")
    sgq.fermi_level(plan, tw, w, 1.0, P.kT, res)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_ENONFINITE
    assert np.isnan(res[0].item())
    announce("node over the atom limit: adjoint")
    dV, dR, dE = sgq.energy_backward(P, sgq.SGQ_FREE, 1.0, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_ELIMIT
    rdV, rdE, rdR = O.band_energy_backward(far, kind=O.FREE)
    assert O.normwise_rel_err(dV.cpu().numpy(), rdV) < 1e-6
    assert not torch.any(dR) and not torch.any(dE) and not np.any(rdR) and not np.any(rdE)
    plan.close()


def test_host_checks_of_compute_calls():
    """Calls the host rejects before launching anything: SGQ_EPLAN for a Gauss rule from the
    plain schedule and for a backward before sgq_plan_prepare_backward, SGQ_EINVAL for
    kT <= 0 or a non-finite mu.  The plan stays usable and matches the oracle after."""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2, grid=32, n_nodes=2)
    P.half_width[:] = 4
    P.depth[:] = 10
    plan = sgq.Plan.from_problem(P)
    v, R, E, w = sgq.device_inputs(P)
    rho = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    tw = torch.zeros(P.n_nodes * plan.kmax * 2, dtype=torch.float64, device="cuda")
    announce("host checks: rejected calls")
    for mu, kT in ((P.mu, 0.0), (P.mu, -1.0), (float("nan"), P.kT), (P.mu, float("inf"))):
        with pytest.raises(sgq.SgqError) as err:
            sgq.rho_quadrature(plan, v, R, E, mu, kT, rho)
        assert err.value.code == sgq.SGQ_EINVAL
    plan.set_schedule(sgq.SGQ_SCHEDULE_PLAIN)
    with pytest.raises(sgq.SgqError) as err:
        sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho, tw)
    assert err.value.code == sgq.SGQ_EPLAN
    plan.set_schedule(sgq.SGQ_SCHEDULE_BATCHED)
    sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    ref, _ = O.rho_quadrature(P)
    assert O.normwise_rel_err(rho.cpu().numpy(), ref) < 1e-4
    g = torch.ones(1, dtype=torch.float64, device="cuda")
    dV = torch.empty_like(v)
    dR = torch.zeros_like(R)
    announce("host checks: backward before its workspace is prepared")
    with pytest.raises(sgq.SgqError) as err:
        sgq.band_energy_backward(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, g, dV, dR)
    assert err.value.code == sgq.SGQ_EPLAN
    plan.prepare_backward()
    plan.prepare_backward()   # a second call is a no-op
    sgq.band_energy_backward(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, g, dV, dR)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    rdV, _, rdR = O.band_energy_backward(P, kind=O.FREE)
    assert O.normwise_rel_err(dV.cpu().numpy(), rdV) < 1e-4
    plan.close()
