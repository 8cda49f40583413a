"""The allocation-free Fermi-level entry point (sgq_fermi_level_noalloc) against the plan's
sgq_fermi_level, through the C ABI: two calls in a row, the second on a smaller input, and the
error code of an unreachable electron count.  Collected last: the entry point's state lives in
a device array that every call on the GPU shares."""
import numpy as np
import pytest

from paper_1907_02604_amd import synth
from gpu_util import announce, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def _noalloc(sgq):
    """The entry point with the arguments in C order; returns its status code."""
    def call(tw, w, n_nodes, kmax, ne, kT, tol, result, status, stream):
        return sgq.fermi_level_noalloc(tw, w, n_nodes, kmax, ne, kT, result, status, tol=tol,
                                       stream=stream)
    return call


def _rules(sgq, prob):
    import torch
    plan = sgq.Plan.from_problem(prob)
    rho, tw, _ = sgq.rho(prob, plan=plan, want_rule=True)
    w = torch.as_tensor(prob.weight, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    ne = float((w * rho).sum().item()) * prob.h ** 3
    return plan, tw.contiguous(), w, ne


def test_noalloc_fermi_level_matches_the_plan_entry_point():
    import torch
    from paper_1907_02604_amd import sgq
    f = _noalloc(sgq)
    big = synth.make_problem(2, grid=32, n_nodes=96)
    big.half_width[:] = 6
    big.depth[:] = 24
    small = big.subset(np.arange(40))
    stream = torch.cuda.current_stream().cuda_stream
    for prob, tag in ((big, "96 nodes"), (small, "40 nodes")):
        announce(f"no-alloc Fermi level, {tag}")
        plan, tw, w, ne = _rules(sgq, prob)
        ref = torch.zeros(3, dtype=torch.float64, device="cuda")
        sgq.fermi_level(plan, tw, w, ne, prob.kT, ref, tol=1e-12)
        got = torch.full((3,), -7.0, dtype=torch.float64, device="cuda")
        code = torch.full((1,), 99, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        st = f(tw, w, prob.n_nodes, plan.kmax, ne, prob.kT, 1e-12, got, code, stream)
        assert st == sgq.SGQ_OK, sgq.lib().sgq_last_error().decode()
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free0
        assert plan.status() == sgq.SGQ_OK
        assert int(code.item()) == sgq.SGQ_OK
        r, g = ref.cpu().numpy(), got.cpu().numpy()
        print(tag, "plan", r, "no-alloc", g)
        assert np.array_equal(r, g)              # same kernels, same order: bitwise equal
        assert abs(g[1] - ne) <= 1e-10 * ne      # the level holds the requested count
        plan.close()


def test_noalloc_fermi_level_errors():
    import torch
    from paper_1907_02604_amd import sgq
    f = _noalloc(sgq)
    prob = synth.make_problem(2, grid=32, n_nodes=8)
    prob.half_width[:] = 4
    prob.depth[:] = 12
    plan, tw, w, ne = _rules(sgq, prob)
    got = torch.zeros(3, dtype=torch.float64, device="cuda")
    code = torch.zeros(1, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    announce("no-alloc Fermi level, unreachable count")
    total = 2.0 * float(w.sum().item())
    assert f(tw, w, prob.n_nodes, plan.kmax, 2.0 * total, prob.kT, 1e-12, got, code,
             stream) == sgq.SGQ_OK
    torch.cuda.synchronize()
    assert int(code.item()) == sgq.SGQ_ERANGE and np.isnan(got[0].item())
    # host-side argument checks return before any launch
    assert f(tw, w, 0, plan.kmax, ne, prob.kT, 1e-12, got, code, stream) == sgq.SGQ_EINVAL
    assert f(tw, w, 1 << 24, 128, ne, prob.kT, 1e-12, got, code, stream) == sgq.SGQ_EINVAL
    assert f(None, w, prob.n_nodes, plan.kmax, ne, prob.kT, 1e-12, got, code, stream) == sgq.SGQ_EINVAL
    assert f(tw, w, prob.n_nodes, plan.kmax, ne, 0.0, 1e-12, got, code, stream) == sgq.SGQ_EINVAL
    # a later good call still works (the error left nothing behind)
    announce("no-alloc Fermi level after an error")
    assert f(tw, w, prob.n_nodes, plan.kmax, ne, prob.kT, 1e-12, got, code, stream) == sgq.SGQ_OK
    torch.cuda.synchronize()
    assert int(code.item()) == sgq.SGQ_OK and abs(got[1].item() - ne) <= 1e-10 * ne
    plan.close()
