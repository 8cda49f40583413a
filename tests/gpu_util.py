"""Helpers of the GPU parity tests (GPU path through the C ABI, oracle on the CPU)."""
import sys

import numpy as np
import pytest

import oracle as O

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:  # pragma: no cover
    HAVE_GPU = False

needs_gpu = pytest.mark.skipif(not HAVE_GPU, reason="no GPU visible")


def announce(msg):
    """Name the case before a GPU step (a fault may end the process)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def gpu_rho(prob, want_rule=False, precision=None):
    from paper_1907_02604_amd import sgq
    prec = {"f64": sgq.SGQ_FP64, "f32": sgq.SGQ_FP32}[precision or prob.precision]
    plan = sgq.Plan(prob.n, prob.h, prob.atoms.shape[0], prob.n_proj, prob.centers,
                    prob.half_width, prob.depth, prec)
    v, R, E, _ = sgq.device_inputs(prob)
    rho = torch.empty(prob.n_nodes, dtype=torch.float64, device="cuda")
    ke = torch.zeros(prob.n_nodes, dtype=torch.int32, device="cuda")
    tw = torch.zeros(prob.n_nodes * plan.kmax * 2, dtype=torch.float64, device="cuda") if want_rule else None
    sgq.rho_quadrature(plan, v, R, E, prob.mu, prob.kT, rho, tw, ke)
    torch.cuda.synchronize()
    status = plan.status()
    out = (rho.cpu().numpy(), ke.cpu().numpy(), status)
    if want_rule:
        out = out + (tw.view(prob.n_nodes, plan.kmax, 2).cpu().numpy(),)
    plan.close()
    return out


def gpu_rho_bench_launch(prob, tune_nodes=2048):
    """rho of `prob` in the launch configuration the benchmark times: the autotuned shape,
    on a side stream, captured into a HIP graph on the first call and replayed on the
    second (the replay's result is returned).  Returns (rho, k_eff, status, shape)."""
    from paper_1907_02604_amd import sgq
    plan = sgq.Plan.from_problem(prob)
    v, R, E, _ = sgq.device_inputs(prob)
    side = torch.cuda.Stream()
    shape = plan.autotune(v, R, E, prob.mu, prob.kT, sample_nodes=tune_nodes,
                          stream=side.cuda_stream)
    rho = torch.empty(prob.n_nodes, dtype=torch.float64, device="cuda")
    ke = torch.zeros(prob.n_nodes, dtype=torch.int32, device="cuda")
    for _ in range(2):
        rho.fill_(-1.0)
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            sgq.rho_quadrature(plan, v, R, E, prob.mu, prob.kT, rho, None, ke,
                               stream=side.cuda_stream)
        side.synchronize()
    status = plan.status()
    out = (rho.cpu().numpy(), ke.cpu().numpy(), status, shape)
    plan.close()
    return out


def gpu_energy(prob, kind, precision=None):
    from paper_1907_02604_amd import sgq
    prec = {"f64": sgq.SGQ_FP64, "f32": sgq.SGQ_FP32}[precision or prob.precision]
    plan = sgq.Plan(prob.n, prob.h, prob.atoms.shape[0], prob.n_proj, prob.centers,
                    prob.half_width, prob.depth, prec)
    v, R, E, w = sgq.device_inputs(prob)
    e = torch.empty(prob.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    sgq.band_energy(plan, v, R, E, w, prob.mu, prob.kT, kind, e, om)
    torch.cuda.synchronize()
    assert plan.status() == 0
    plan.close()
    return e.cpu().numpy(), float(om.item())


def oracle_rho(prob, nodes):
    return O.rho_quadrature(prob, nodes=nodes)


def stratified_sample(prob, count, seed):
    """Nodes spread over the cost range (cube size x depth), seeded."""
    cost = (2 * prob.half_width.astype(np.float64) + 1) ** 3 * prob.depth
    order = np.argsort(cost, kind="stable")
    rng = np.random.default_rng(seed)
    bins = np.array_split(order, count)
    return np.array([rng.choice(b) for b in bins if b.size], dtype=np.int64)
