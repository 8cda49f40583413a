"""The compute calls allocate nothing and do not synchronise: their workspace comes from the
set-up calls (sgq_plan_create, sgq_plan_prepare_backward, sgq_plan_set_schedule)."""
import numpy as np
import pytest

import oracle as O
from paper_1907_02604_amd import synth
from gpu_util import announce, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def test_first_backward_runs_beside_other_work_without_a_sync():
    """A long forward launch runs on one stream; the first band_energy_backward of another,
    prepared plan is enqueued on a second stream.  The call returns while the first stream
    is still busy (no device synchronisation), the free device memory is unchanged across it
    (no allocation), and its gradient matches the oracle.  (The HIP runtime sets up a
    stream's own buffers, such as kernel arguments and spill scratch, on its first launches:
    a backward of a third plan on that stream comes first, so that only the library's own
    allocations would show.)"""
    import torch
    from paper_1907_02604_amd import sgq
    big = synth.make_problem(2, n_nodes=4096)
    bplan = sgq.Plan.from_problem(big)
    bv, bR, bE, _ = sgq.device_inputs(big)
    brho = torch.empty(big.n_nodes, dtype=torch.float64, device="cuda")
    small = synth.make_problem(4).subset(np.random.default_rng(5).choice(110592, 3, replace=False))
    splan = sgq.Plan.from_problem(small)
    splan.prepare_backward()
    v, R, E, w = sgq.device_inputs(small)
    g = torch.ones(1, dtype=torch.float64, device="cuda")
    dV = torch.empty_like(v)
    dR = torch.zeros_like(R)
    dE = torch.zeros_like(E)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    done = torch.cuda.Event()
    announce("alloc-free: warm-up forward of the long plan, warm-up backward of a third plan")
    with torch.cuda.stream(sa):
        sgq.rho_quadrature(bplan, bv, bR, bE, big.mu, big.kT, brho, stream=sa.cuda_stream)
    other = synth.make_problem(4).subset([17, 4242])
    oplan = sgq.Plan.from_problem(other)
    oplan.prepare_backward()
    ov, oR, oE, ow = sgq.device_inputs(other)
    odV, odR, odE = torch.empty_like(ov), torch.zeros_like(oR), torch.zeros_like(oE)
    with torch.cuda.stream(sb):
        sgq.band_energy_backward(oplan, ov, oR, oE, ow, other.mu, other.kT, sgq.SGQ_FREE, g, odV,
                                 odR, odE, stream=sb.cuda_stream)
    torch.cuda.synchronize()
    assert oplan.status() == sgq.SGQ_OK
    free0 = torch.cuda.mem_get_info()[0]
    announce("alloc-free: long forward on one stream, first backward on another")
    with torch.cuda.stream(sa):
        sgq.rho_quadrature(bplan, bv, bR, bE, big.mu, big.kT, brho, stream=sa.cuda_stream)
        done.record(sa)
    with torch.cuda.stream(sb):
        sgq.band_energy_backward(splan, v, R, E, w, small.mu, small.kT, sgq.SGQ_FREE, g, dV, dR,
                                 dE, stream=sb.cuda_stream)
    busy = not done.query()
    free1 = torch.cuda.mem_get_info()[0]
    torch.cuda.synchronize()
    assert busy, "the long forward finished before the backward call returned"
    assert free1 == free0
    assert splan.status() == sgq.SGQ_OK
    rdV, rdE, rdR = O.band_energy_backward(small, kind=O.FREE)
    for got, ref in ((dV, rdV), (dR, rdR), (dE, rdE)):
        assert O.normwise_rel_err(got.cpu().numpy(), ref) < 1e-4
    bplan.close()
    splan.close()
    oplan.close()


def test_plain_schedule_scratch_is_set_up_by_set_schedule():
    """sgq_plan_set_schedule(PLAIN) allocates the plain schedule's scratch; its density calls
    then leave the free device memory unchanged and match the oracle.  (The first call comes
    before the measurement: the HIP runtime sets up a kernel's private memory on its first
    launch.)"""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2, grid=32, n_nodes=3)
    P.half_width[:] = 5
    P.depth[:] = 14
    plan = sgq.Plan.from_problem(P)
    v, R, E, _ = sgq.device_inputs(P)
    rho = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    plan.set_schedule(sgq.SGQ_SCHEDULE_PLAIN)
    announce("alloc-free: plain schedule density, first call")
    sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    announce("alloc-free: plain schedule density")
    for _ in range(2):
        sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
    assert plan.status() == sgq.SGQ_OK
    ref, _ = O.rho_quadrature(P)
    assert O.normwise_rel_err(rho.cpu().numpy(), ref) < 1e-4
    plan.close()
