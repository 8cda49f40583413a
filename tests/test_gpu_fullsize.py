"""Full-size launches of the two largest workloads, checked where the oracle cannot run them
whole: sampled nodes against the oracle, and properties that hold at any size (linearity of
the adjoint in the node weights, the adjoint against central differences of the full-size
energy)."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from oracle_util import oracle_rho_pool, per_node_rel_err, smooth_random_potential
from paper_1907_02604_amd import synth
from gpu_util import announce, gpu_rho_bench_launch, needs_gpu, stratified_sample

pytestmark = [pytest.mark.gpu, needs_gpu]


def _grad(P, plan, kind):
    import torch
    from paper_1907_02604_amd import sgq
    dV, dR, dE = sgq.energy_backward(P, kind, 1.0, plan=plan)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    return dV.cpu().numpy(), dR.cpu().numpy(), dE.cpu().numpy()


def test_dislocation_workload_all_65536_nodes():
    """128^3 screw lattice, all 65536 nodes (cubes 25^3..49^3, K = 80, weights 32), FP32, in
    the autotuned launch: 48 stratified nodes against the oracle; the adjoint of all nodes
    equals the sum of the adjoints of the two halves of the node list (the gather over
    65536 node cubes against two gathers over 32768)."""
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(5)
    assert P.n_nodes == 65536
    announce("C5 full: forward, 65536 nodes, benchmark launch")
    rho, _, st, shape = gpu_rho_bench_launch(P)
    print("C5 launch shape", shape)
    assert st == sgq.SGQ_OK
    sample = stratified_sample(P, 48, seed=31)
    ref = oracle_rho_pool(P, sample)
    err = O.normwise_rel_err(rho[sample], ref)
    pn = per_node_rel_err(rho[sample], ref)
    print("C5 full forward sampled err", err, "per node", pn)
    assert err < 1e-4
    assert pn < 1e-4 / 1e-3
    plan = sgq.Plan.from_problem(P)
    announce("C5 full: adjoint, 65536 nodes")
    full = _grad(P, plan, sgq.SGQ_FREE)
    plan.close()
    half = np.arange(P.n_nodes) % 2 == 0
    parts = []
    for sel in (half, ~half):
        Q = P.subset(np.nonzero(sel)[0])
        qplan = sgq.Plan.from_problem(Q)
        announce(f"C5 full: adjoint of {Q.n_nodes} nodes")
        parts.append(_grad(Q, qplan, sgq.SGQ_FREE))
        qplan.close()
    for a, b, c, name in zip(full, parts[0], parts[1], ("dV", "dR", "dE")):
        e = O.normwise_rel_err(a, b + c)
        print("C5 linearity", name, e)
        assert e < 1e-6, name


def test_differentiation_workload_all_nodes_central_difference():
    """48^3 grid, all 110592 nodes, FP64: the adjoint's dOmega/dV along a smooth random
    direction d against (Omega(V + eps d) - Omega(V - eps d)) / (2 eps) of the full-size
    band free energy, eps = 1e-4 (the workload's step).  Then the FP32 adjoint of all nodes
    against that FP64 adjoint: dV, dR and dE within 1e-4."""
    import torch
    from paper_1907_02604_amd import sgq
    P = dataclasses.replace(synth.make_problem(4), precision="f64")
    assert P.n_nodes == 110592
    plan = sgq.Plan.from_problem(P)
    announce("C4 full fp64: adjoint, 110592 nodes")
    dV, dR, dE = _grad(P, plan, sgq.SGQ_FREE)
    d = smooth_random_potential(48, seed=5)
    eps = 1e-4
    om = []
    for sgn in (1.0, -1.0):
        Pp = dataclasses.replace(P, v_loc=P.v_loc + sgn * eps * d)
        v, R, E, w = sgq.device_inputs(Pp)
        e = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
        o = torch.empty(1, dtype=torch.float64, device="cuda")
        announce(f"C4 full fp64: forward at V {'+' if sgn > 0 else '-'} eps d")
        sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, o)
        torch.cuda.synchronize()
        assert plan.status() == sgq.SGQ_OK
        om.append(o.item())
    fd = (om[0] - om[1]) / (2 * eps)
    an = float(np.sum(dV * d))
    print("C4 full central difference", fd, "adjoint", an)
    assert abs(fd - an) <= 1e-6 * abs(an)
    plan.close()
    P32 = dataclasses.replace(P, precision="f32")
    plan32 = sgq.Plan.from_problem(P32)
    announce("C4 full fp32: adjoint, 110592 nodes")
    g32 = _grad(P32, plan32, sgq.SGQ_FREE)
    plan32.close()
    for a, b, name in zip(g32, (dV, dR, dE), ("dV", "dR", "dE")):
        e = O.normwise_rel_err(a, b)
        print("C4 full fp32 vs fp64 adjoint", name, e)
        assert e < 1e-4, name
