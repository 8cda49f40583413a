"""Retained forward bases (sgq_plan_set_retain): the backward that takes them gives bitwise
the gradient of the backward that recomputes them, and the retention is consumed, keyed to
the input pointers and invalidated by other forward launches."""
import numpy as np
import pytest

from paper_1907_02604_amd import synth
from gpu_util import announce, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def _forward_backward(plan, P, v, R, E, w):
    import torch
    from paper_1907_02604_amd import sgq
    e = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
    g = _backward(plan, P, v, R, E, w)
    return (e.cpu().numpy(),) + g


def _backward(plan, P, v, R, E, w):
    import torch
    from paper_1907_02604_amd import sgq
    g = torch.ones(1, dtype=torch.float64, device="cuda")
    dV = torch.empty_like(v)
    dR = torch.zeros_like(R)
    dE = torch.zeros_like(E)
    sgq.band_energy_backward(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, g, dV, dR, dE)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    return dV.cpu().numpy(), dR.cpu().numpy(), dE.cpu().numpy()


@pytest.mark.parametrize("precision", ["f32", "f64"])
def test_retained_backward_is_bitwise_the_recompute(precision):
    import dataclasses
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(4)
    P = dataclasses.replace(P.subset(np.random.default_rng(3).choice(P.n_nodes, 96, replace=False)),
                            precision=precision)
    v, R, E, w = sgq.device_inputs(P)
    announce(f"retain {precision}: recompute path")
    plain = sgq.Plan.from_problem(P)
    ref = _forward_backward(plain, P, v, R, E, w)
    plain.close()
    announce(f"retain {precision}: retained path")
    plan = sgq.Plan.from_problem(P)
    plan.set_retain(True)
    got = _forward_backward(plan, P, v, R, E, w)
    for a, b, name in zip(ref, got, ("e_node", "dV", "dR", "dE")):
        assert np.array_equal(a, b), name
    # consumed: the next backward recomputes, with the same result
    announce(f"retain {precision}: second backward (recompute)")
    again = _backward(plan, P, v, R, E, w)
    for a, b in zip(ref[1:], again):
        assert np.array_equal(a, b)
    plan.close()


def test_retention_is_keyed_to_the_inputs_and_invalidated():
    """A forward with other input pointers, or an autotune in between, leaves the backward
    to recompute: the gradients stay those of the backward's own inputs."""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(4)
    P = P.subset(np.random.default_rng(4).choice(P.n_nodes, 64, replace=False))
    v, R, E, w = sgq.device_inputs(P)
    plan = sgq.Plan.from_problem(P)
    announce("retain keys: reference")
    ref = _backward(plan, P, v, R, E, w)          # nothing retained yet: recompute
    plan.set_retain(True)
    v2 = (v * 1.01).contiguous()                  # other inputs
    e = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    announce("retain keys: forward on other inputs, backward on the first")
    sgq.band_energy(plan, v2, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
    got = _backward(plan, P, v, R, E, w)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    announce("retain keys: forward, autotune, backward")
    sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
    plan.autotune(v, R, E, P.mu, P.kT, sample_nodes=16)
    got = _backward(plan, P, v, R, E, w)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    plan.close()
