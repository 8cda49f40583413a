"""The adjoint's eigensolve pre-pass: when a plan's last forward launch stored every node's
tridiagonal for the same inputs, the backward takes the eigensolves and Daleckii-Krein
steps from a pass of their own; otherwise it solves in place.  Both use the same code, so on
the same tridiagonal they give the same bits; a forward with another launch shape stores a
tridiagonal that differs from the backward's recompute in the last bits, which shows that
the pass ran, within the FP32 bar of the recompute's gradient."""
import numpy as np
import pytest

from paper_1907_02604_amd import synth
from gpu_util import announce, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def _problem(precision="f32", n=40, seed=12, cfg=4):
    """n seeded nodes of the workload; of the dislocation workload only cubes of at most 35
    points, which the backward reverses with the default forward's 256 lanes."""
    import dataclasses
    P = synth.make_problem(cfg)
    pool = np.nonzero(2 * P.half_width + 1 <= 35)[0]
    P = P.subset(np.sort(np.random.default_rng(seed).choice(pool, n, replace=False)))
    return dataclasses.replace(P, precision=precision)


def _backward(plan, P, v, R, E, w, forward_first):
    """(dV, dR, dE) on host; the forward band_energy call first when asked (same tensors,
    so the plan's stored tridiagonals belong to these inputs)."""
    import torch
    from paper_1907_02604_amd import sgq
    plan.prepare_backward()
    if forward_first:
        e = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
        om = torch.empty(1, dtype=torch.float64, device="cuda")
        sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
    g = torch.ones(1, dtype=torch.float64, device="cuda")
    dV = torch.empty_like(v)
    dR = torch.zeros_like(R)
    dE = torch.zeros_like(E)
    sgq.band_energy_backward(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, g, dV, dR, dE)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    return dV.cpu().numpy(), dR.cpu().numpy(), dE.cpu().numpy()


@pytest.mark.parametrize("cfg,precision", [(4, "f32"), (4, "f64"), (5, "f32")])
def test_prepass_gives_the_in_place_solve_bit_for_bit(cfg, precision):
    """A forward then a backward (pre-pass over the forward's tridiagonals) against a
    backward alone (eigensolves in place), both with the default 256-lane forward: same
    bits, at K = 60 (differentiation workload) and K = 80 (dislocation workload, cubes of
    25^3..33^3)."""
    from paper_1907_02604_amd import sgq
    P = _problem(precision, n=40 if cfg == 4 else 12, cfg=cfg)
    v, R, E, w = sgq.device_inputs(P)
    announce(f"prepass {precision}: forward + backward")
    plan = sgq.Plan.from_problem(P)
    got = _backward(plan, P, v, R, E, w, forward_first=True)
    plan.close()
    announce(f"prepass {precision}: backward alone")
    plan = sgq.Plan.from_problem(P)
    ref = _backward(plan, P, v, R, E, w, forward_first=False)
    plan.close()
    for a, b, name in zip(got, ref, ("dV", "dR", "dE")):
        assert np.array_equal(a, b), name


def test_prepass_takes_the_forward_tridiagonal(monkeypatch):
    """After a 128-lane forward (another autotuner candidate; the backward recomputes these
    33^3 cubes with 256 lanes whatever the forward's shape) the pre-pass solves the forward's
    tridiagonals,
    whose last bits differ from the recompute's: the gradient is not the in-place one bit
    for bit (so the pass ran) and agrees with it to the FP32 bar."""
    from paper_1907_02604_amd import sgq
    P = _problem("f32", n=48, seed=13)
    v, R, E, w = sgq.device_inputs(P)
    announce("prepass: backward alone")
    plan = sgq.Plan.from_problem(P)
    ref = _backward(plan, P, v, R, E, w, forward_first=False)
    plan.close()
    monkeypatch.setenv("SGQ_BLOCK", "128")
    monkeypatch.setenv("SGQ_WG_PER_CU", "2")
    plan = sgq.Plan.from_problem(P)
    monkeypatch.delenv("SGQ_BLOCK")
    monkeypatch.delenv("SGQ_WG_PER_CU")
    announce("prepass: 128-lane forward + backward")
    got = _backward(plan, P, v, R, E, w, forward_first=True)
    plan.close()
    assert any(not np.array_equal(a, b) for a, b in zip(got, ref))
    for a, b, name in zip(got, ref, ("dV", "dR", "dE")):
        err = np.max(np.abs(a - b)) / np.max(np.abs(b))
        print("prepass vs in place", name, err)
        assert err <= 1e-4, (name, err)


def test_prepass_skips_stale_tridiagonals():
    """The stored tridiagonals serve only the inputs the forward saw: after v_loc is
    overwritten in place (same pointer, new contents), and after autotuning (whose timing
    launches rewrite the sampled nodes' tridiagonals), the backward equals a backward alone
    on the current inputs with the same launch shape, bit for bit."""
    import torch
    from paper_1907_02604_amd import sgq
    P = _problem("f32", n=40, seed=14)
    v, R, E, w = sgq.device_inputs(P)
    plan = sgq.Plan.from_problem(P)
    plan.prepare_backward()
    e = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    announce("prepass stale: forward, then v_loc changed in place")
    sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
    torch.cuda.synchronize()
    v.mul_(1.01)
    got = _backward(plan, P, v, R, E, w, forward_first=False)
    fresh = sgq.Plan.from_problem(P)
    ref = _backward(fresh, P, v, R, E, w, forward_first=False)
    fresh.close()
    for a, b, name in zip(got, ref, ("dV", "dR", "dE")):
        assert np.array_equal(a, b), ("in-place change", name)
    announce("prepass stale: forward, then autotune")
    sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
    plan.autotune(v, R, E, P.mu, P.kT, sample_nodes=16)
    got = _backward(plan, P, v, R, E, w, forward_first=False)
    plan.close()
    # the same as a fresh plan's: the backward's lanes per node follow the node's cube, not
    # the autotuned shape
    fresh = sgq.Plan.from_problem(P)
    ref = _backward(fresh, P, v, R, E, w, forward_first=False)
    fresh.close()
    for a, b, name in zip(got, ref, ("dV", "dR", "dE")):
        assert np.array_equal(a, b), ("autotune", name)
