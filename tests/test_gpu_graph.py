"""Captured launch sequences (HIP graphs) and the launch-shape autotuner, on the GPU.

Graph replays are compared bit for bit with direct launches of the same plan shape, with
eager device work and synchronisations between the replays; the autotuned launch shape
is checked against the FP64 oracle."""
import numpy as np
import pytest

import oracle as O
from paper_1907_02604_amd import synth
from gpu_util import announce, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def _plan(P, graph):
    from paper_1907_02604_amd import sgq
    plan = sgq.Plan.from_problem(P)
    plan.set_graph(graph)
    return plan


def test_graph_replays_match_direct_launches():
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2).subset(np.arange(256))
    v, R, E, w = sgq.device_inputs(P)
    announce("graph: direct launches, 256 C2 nodes")
    direct = _plan(P, False)
    rho0 = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    e0 = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    om0 = torch.empty(1, dtype=torch.float64, device="cuda")
    sgq.rho_quadrature(direct, v, R, E, P.mu, P.kT, rho0)
    sgq.band_energy(direct, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e0, om0)
    rho_mu = torch.empty_like(rho0)
    sgq.rho_quadrature(direct, v, R, E, P.mu + 0.05, P.kT, rho_mu)
    torch.cuda.synchronize()
    assert direct.status() == 0

    announce("graph: captured launches on a side stream")
    plan = _plan(P, True)
    side = torch.cuda.Stream()
    rho = torch.empty_like(rho0)
    e = torch.empty_like(e0)
    om = torch.empty_like(om0)
    scratch = torch.randn(1 << 20, device="cuda")
    for rep in range(4):
        rho.fill_(-1.0)
        e.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho, stream=side.cuda_stream)
            sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, om,
                            stream=side.cuda_stream)
        side.synchronize()
        scratch.mul_(1.0001).add_(0.5)      # eager work between the replays
        torch.cuda.synchronize()
        assert plan.status() == 0
        assert torch.equal(rho, rho0), f"replay {rep}: rho differs from the direct launch"
        assert torch.equal(e, e0), f"replay {rep}: e_node differs"
        assert torch.equal(om, om0), f"replay {rep}: omega differs"
    # a changed scalar argument re-captures
    with torch.cuda.stream(side):
        sgq.rho_quadrature(plan, v, R, E, P.mu + 0.05, P.kT, rho, stream=side.cuda_stream)
    side.synchronize()
    assert torch.equal(rho, rho_mu)
    # and the first capture's arguments again
    with torch.cuda.stream(side):
        sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho, stream=side.cuda_stream)
    side.synchronize()
    assert torch.equal(rho, rho0)
    plan.close()
    direct.close()


def test_autotuned_launch_shape_matches_oracle():
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2).subset(np.arange(1536))
    v, R, E, _ = sgq.device_inputs(P)
    plan = sgq.Plan.from_problem(P)
    rho_a = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    announce("autotune: default shape, 1536 C2 nodes")
    sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho_a)
    torch.cuda.synchronize()
    announce("autotune: timing candidates on 768 nodes")
    block, wpc = plan.autotune(v, R, E, P.mu, P.kT, sample_nodes=768)
    print("autotuned shape", block, wpc)
    assert (block, wpc) in {(256, 2), (256, 1), (128, 3), (128, 2), (512, 1)}
    # the cached choice is returned without timing again
    assert plan.autotune(v, R, E, P.mu, P.kT, sample_nodes=768) == (block, wpc)
    rho_b = torch.empty_like(rho_a)
    announce("autotune: tuned shape")
    sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho_b)
    torch.cuda.synchronize()
    assert plan.status() == 0
    a, b = rho_a.cpu().numpy(), rho_b.cpu().numpy()
    assert O.normwise_rel_err(b, a) < 1e-6
    sample = np.random.default_rng(31).choice(P.n_nodes, 8, replace=False)
    ref, _ = O.rho_quadrature(P, nodes=sample)
    err = O.normwise_rel_err(b[sample], ref)
    print("autotuned err vs oracle", err)
    assert err < 1e-4
    plan.close()
