"""Retained forward bases (sgq_plan_set_retain): the backward that takes them gives bitwise
the gradient of the backward that recomputes them, for every node or for the costliest
nodes within a byte limit, and the retention is consumed, keyed to the input pointers and
invalidated by other forward launches."""
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
    plan.prepare_backward()
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
    to recompute: the gradients stay those of the backward's own inputs, bit for bit (the
    backward's lanes per node follow the node's cube, not the autotuned shape)."""
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


def test_inputs_overwritten_in_place_are_detected():
    """The forward retains the bases, the caller then overwrites v_loc in place (same
    pointer, new contents) or a projector energy, and calls the backward: the content hashes
    differ, so the backward recomputes and returns the gradient of the new inputs, bitwise
    that of a plan that never retained anything."""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(4)
    P = P.subset(np.random.default_rng(6).choice(P.n_nodes, 32, replace=False))
    v, R, E, w = sgq.device_inputs(P)
    e = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    plan = sgq.Plan.from_problem(P)
    plan.set_retain(True)
    for what in ("v_loc", "proj_E"):
        announce(f"retain hash: forward, {what} overwritten in place, backward")
        sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
        if what == "v_loc":
            v.mul_(1.02)
        else:
            E[0, 1] += 0.05
        got = _backward(plan, P, v, R, E, w)
        fresh = sgq.Plan.from_problem(P)
        ref = _backward(fresh, P, v, R, E, w)
        fresh.close()
        for a, b in zip(ref, got):
            assert np.array_equal(a, b)
    announce("retain hash: unchanged inputs take the retained rows")
    sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, sgq.SGQ_FREE, e, om)
    got = _backward(plan, P, v, R, E, w)
    fresh = sgq.Plan.from_problem(P)
    ref = _backward(fresh, P, v, R, E, w)
    fresh.close()
    for a, b in zip(ref, got):   # the same launch shape: the retained rows are bitwise the recompute's
        assert np.array_equal(a, b)
    plan.close()


def test_retention_within_a_byte_limit_keeps_the_costliest_nodes():
    """Dislocation-shaped nodes with cubes of 25^3, 29^3 and 33^3 (K = 80; the backward reverses
    them with 256 lanes, as the default forward runs them): a limit that holds a third of
    the nodes' rows retains that many, the backward takes them and recomputes the rest, and
    the gradient is bitwise the full recompute's.  A limit below one node is rejected."""
    from paper_1907_02604_amd import sgq
    P5 = synth.make_problem(5)
    narrow = np.nonzero(2 * P5.half_width + 1 <= 35)[0]
    P = P5.subset(np.sort(np.random.default_rng(5).choice(narrow, 36, replace=False)))
    assert len(set(P.half_width.tolist())) == 3
    v, R, E, w = sgq.device_inputs(P)
    announce("retain limit: recompute reference")
    ref_plan = sgq.Plan.from_problem(P)
    ref = _forward_backward(ref_plan, P, v, R, E, w)
    ref_plan.close()
    plan = sgq.Plan.from_problem(P)
    npad = (max((2 * int(r) + 1) ** 3 for r in P.half_width) + 63) // 64 * 64
    per_node = 2 * plan.kmax * npad * 4               # basis and u_j rows, FP32
    with pytest.raises(sgq.SgqError):
        plan.set_retain(True, max_bytes=per_node - 1)
    budget = 12 * per_node + per_node // 2
    assert plan.set_retain(True, max_bytes=budget) == 12
    announce("retain limit: 12 of 36 nodes retained")
    got = _forward_backward(plan, P, v, R, E, w)
    for a, b, name in zip(ref, got, ("e_node", "dV", "dR", "dE")):
        assert np.array_equal(a, b), name
    assert plan.set_retain(True, max_bytes=10 ** 15) == P.n_nodes   # capped at the node count
    assert plan.set_retain(False) == 0
    announce("retain limit: retention off")
    got = _forward_backward(plan, P, v, R, E, w)
    for a, b in zip(ref, got):
        assert np.array_equal(a, b)
    plan.close()


def test_retained_rows_of_another_launch_shape_agree_within_rounding(monkeypatch):
    """A forward with 512 lanes per node (an autotuned shape) sums its sweeps in another
    order than a 256-lane plan's forward and recompute, so its retained rows differ from
    theirs by rounding: the gradient agrees with the 256-lane one to the FP32 bar, 1e-4
    normwise."""
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(4)
    P = P.subset(np.random.default_rng(6).choice(P.n_nodes, 48, replace=False))
    v, R, E, w = sgq.device_inputs(P)
    announce("retain shape: recompute reference (256 lanes)")
    ref_plan = sgq.Plan.from_problem(P)
    ref = _forward_backward(ref_plan, P, v, R, E, w)
    ref_plan.close()
    monkeypatch.setenv("SGQ_BLOCK", "512")         # the autotuner's 512 lanes x 1 per CU
    monkeypatch.setenv("SGQ_WG_PER_CU", "1")
    plan = sgq.Plan.from_problem(P)
    monkeypatch.delenv("SGQ_BLOCK")
    monkeypatch.delenv("SGQ_WG_PER_CU")
    plan.set_retain(True)
    announce("retain shape: 512-lane forward, retained backward")
    got = _forward_backward(plan, P, v, R, E, w)
    plan.close()
    for a, b, name in zip(ref, got, ("e_node", "dV", "dR", "dE")):
        err = np.max(np.abs(a - b)) / np.max(np.abs(a))
        assert err <= 1e-4, (name, err)


def test_retained_wide_nodes_of_a_256_lane_forward_agree_within_rounding():
    """Dislocation nodes with cubes of 25^3..49^3 after a default (256-lane) forward that
    retained them all: the backward reverses the cubes wider than 35 points with 512 lanes,
    whose sweeps sum in another order than the forward's, so the gradient agrees with the
    full recompute's to the FP32 bar, 1e-4 normwise, on every output."""
    from paper_1907_02604_amd import sgq
    P5 = synth.make_problem(5)
    P = P5.subset(np.sort(np.random.default_rng(9).choice(P5.n_nodes, 24, replace=False)))
    assert (2 * P.half_width + 1 > 35).any() and (2 * P.half_width + 1 <= 35).any()
    v, R, E, w = sgq.device_inputs(P)
    announce("retain wide: recompute reference")
    ref_plan = sgq.Plan.from_problem(P)
    ref = _forward_backward(ref_plan, P, v, R, E, w)
    ref_plan.close()
    plan = sgq.Plan.from_problem(P)
    assert plan.set_retain(True) == P.n_nodes
    announce("retain wide: 256-lane forward, retained backward")
    got = _forward_backward(plan, P, v, R, E, w)
    plan.close()
    assert np.array_equal(ref[0], got[0])
    for a, b, name in zip(ref[1:], got[1:], ("dV", "dR", "dE")):
        err = np.max(np.abs(a - b)) / np.max(np.abs(a))
        print("retain wide", name, err)
        assert err <= 1e-4, (name, err)


def test_retention_limits_at_the_edges():
    """FP64 nodes with a limit of exactly one node's rows retain one node and keep the
    recompute's gradient bit for bit; a plan without nodes accepts any limit and retains
    none."""
    import dataclasses
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(4)
    P = dataclasses.replace(P.subset(np.random.default_rng(7).choice(P.n_nodes, 24, replace=False)),
                            precision="f64")
    v, R, E, w = sgq.device_inputs(P)
    announce("retain edges: FP64 recompute reference")
    ref_plan = sgq.Plan.from_problem(P)
    ref = _forward_backward(ref_plan, P, v, R, E, w)
    ref_plan.close()
    plan = sgq.Plan.from_problem(P)
    npad = (max((2 * int(r) + 1) ** 3 for r in P.half_width) + 63) // 64 * 64
    per_node = 2 * plan.kmax * npad * 8               # basis and u_j rows, FP64
    assert plan.set_retain(True, max_bytes=per_node) == 1
    announce("retain edges: one FP64 node retained")
    got = _forward_backward(plan, P, v, R, E, w)
    plan.close()
    for a, b, name in zip(ref, got, ("e_node", "dV", "dR", "dE")):
        assert np.array_equal(a, b), name
    empty = sgq.Plan.from_problem(synth.make_problem(2, grid=32, n_nodes=1).subset([]))
    assert empty.set_retain(True, max_bytes=1) == 0
    assert empty.set_retain(True) == 0
    empty.close()
