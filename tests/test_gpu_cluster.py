"""Cluster-sampled energy (sgq_cluster_build + band_energy + sgq_cluster_energy) on the GPU
against the FP64 oracle's cluster averages."""
import numpy as np
import pytest

import oracle as O
from paper_1907_02604_amd import synth
from gpu_util import announce, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]


def _run(P, esp, radius, esp_weight=None, kind=None):
    """Device cluster energy: returns (node problem, clusters, e_node, fbar, energy, omega)."""
    import torch
    from paper_1907_02604_amd import sgq
    kind = sgq.SGQ_FREE if kind is None else kind
    Pn, cl = sgq.cluster_problem(P, esp, radius, esp_weight)
    plan = sgq.Plan.from_problem(Pn)
    v, R, E, wn = sgq.device_inputs(Pn)
    e = torch.empty(Pn.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    sgq.band_energy(plan, v, R, E, wn, Pn.mu, Pn.kT, kind, e, om)
    off = torch.as_tensor(cl["member_offset"], device="cuda")
    mem = torch.as_tensor(cl["member_node"], device="cuda")
    we = torch.as_tensor(cl["esp_weight"], device="cuda")
    fbar = torch.empty(len(esp), dtype=torch.float64, device="cuda")
    en = torch.empty(1, dtype=torch.float64, device="cuda")
    sgq.cluster_energy(plan, e, off, mem, we, fbar, en)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    plan.close()
    return Pn, cl, e.cpu().numpy(), fbar.cpu().numpy(), en.item(), om.item()


def test_cluster_energy_matches_oracle_with_shared_points():
    """Four ESPs of the 64^3 system, two of them one grid point apart (their balls share
    points), radius 0.5 bohr (7-point balls): Fbar_q and sum_q n_q Fbar_q against the
    oracle's brute-force clusters of oracle energies, at the FP32 path's bar."""
    P = synth.make_problem(2)
    c0 = int(P.centers[0])
    P.centers[1] = c0 + 1 if (c0 + 1) % 64 else c0 - 1
    esp = np.arange(4)
    w = np.array([1.0, 3.0, 0.5, 12.0])
    announce("cluster energy: 4 ESPs of C2, r = 0.5 bohr")
    Pn, cl, e, fbar, energy, omega = _run(P, esp, 0.5, w)
    assert Pn.n_nodes == 4 * 7 - 2          # the two neighbouring balls share two points
    lookup = {int(p): i for i, p in enumerate(Pn.centers)}
    ref_e, _ = O.band_energy(Pn, kind=O.FREE)
    ref_E, ref_fbar = O.cluster_energy(lambda p: ref_e[lookup[p]], P.n, P.h, P.centers[esp], w, 0.5)
    print("fbar", fbar, "oracle", ref_fbar, "E", energy, ref_E)
    assert O.normwise_rel_err(e, ref_e) < 1e-4
    assert O.normwise_rel_err(fbar, ref_fbar) < 1e-4
    assert abs(energy - ref_E) <= 1e-4 * abs(ref_E)
    # the node-weighted band energy with the cluster node weights is the same sum
    assert abs(omega - energy) <= 1e-12 * abs(energy)


def test_cluster_mean_is_exact_and_reproducible():
    """The segmented mean of given energies over clusters longer than a wavefront
    (123-point balls: one full stride of 64 and a ragged one of 59) and a partial last
    workgroup (4097 ESPs): FP64 means within the rounding bound of two 123-term sums in
    different orders, bitwise equal on a second call."""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2)
    rng = np.random.default_rng(7)
    esp_c = rng.choice(64 ** 3, 4097, replace=False)
    cl = sgq.cluster_build(P.n, P.h, esp_c, 1.5)
    nn = cl["node_center"].size
    assert np.all(np.diff(cl["member_offset"]) == 123)
    plan = sgq.Plan(P.n, P.h, 0, 0, cl["node_center"], np.full(nn, 2, np.int32),
                    np.full(nn, 4, np.int32), sgq.SGQ_FP64)
    e_h = rng.normal(size=nn)
    w_h = rng.uniform(0.5, 40.0, size=esp_c.size)
    e = torch.as_tensor(e_h, device="cuda")
    off = torch.as_tensor(cl["member_offset"], device="cuda")
    mem = torch.as_tensor(cl["member_node"], device="cuda")
    we = torch.as_tensor(w_h, device="cuda")
    fbar = torch.empty(esp_c.size, dtype=torch.float64, device="cuda")
    en = torch.empty(1, dtype=torch.float64, device="cuda")
    announce("cluster mean: 4097 clusters of 123 points")
    sgq.cluster_energy(plan, e, off, mem, we, fbar, en)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    f = fbar.cpu().numpy()
    ref = np.array([np.sum(e_h[cl["member_node"][a:b]]) / (b - a)
                    for a, b in zip(cl["member_offset"][:-1], cl["member_offset"][1:])])
    eps = np.finfo(np.float64).eps
    bound = np.array([2 * 122 * eps * np.mean(np.abs(e_h[cl["member_node"][a:b]]))
                      for a, b in zip(cl["member_offset"][:-1], cl["member_offset"][1:])])
    assert np.all(np.abs(f - ref) <= bound)
    assert abs(en.item() - np.dot(w_h, ref)) <= 1e-13 * np.sum(np.abs(w_h * ref))
    f2 = torch.empty_like(fbar)
    en2 = torch.empty_like(en)
    sgq.cluster_energy(plan, e, off, mem, we, f2, en2)
    torch.cuda.synchronize()
    assert torch.equal(fbar, f2) and torch.equal(en, en2)
    # without the weights only the means are written
    f3 = torch.empty_like(fbar)
    sgq.cluster_energy(plan, e, off, mem, None, f3)
    torch.cuda.synchronize()
    assert torch.equal(fbar, f3)
    plan.close()


def test_cluster_list_errors_are_latched():
    """A member outside the plan's nodes, an empty cluster and an offset past the member
    list latch SGQ_EINDEX (their means are NaN, the other clusters are still written); a
    non-finite energy SGQ_ENONFINITE."""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2)
    plan = sgq.Plan(P.n, P.h, 0, 0, np.arange(10, dtype=np.int64), np.full(10, 2, np.int32),
                    np.full(10, 4, np.int32), sgq.SGQ_FP64)
    e = torch.arange(10, dtype=torch.float64, device="cuda")
    fbar = torch.empty(3, dtype=torch.float64, device="cuda")
    announce("cluster lists: an index past the nodes, an empty cluster")
    for off, mem, bad in (([0, 3, 5, 7], [0, 1, 2, 3, 10, 5, 6], 1),
                          ([0, 3, 3, 5], [0, 1, 2, 3, 4], 1),
                          ([0, 3, 5, 9], [0, 1, 2, 3, 4, 5, 6], 2)):
        sgq.cluster_energy(plan, e, torch.tensor(off, device="cuda"),
                           torch.tensor(mem, dtype=torch.int32, device="cuda"), None, fbar)
        torch.cuda.synchronize()
        assert plan.status() == sgq.SGQ_EINDEX
        f = fbar.cpu().numpy()
        assert np.isnan(f[bad]) and f[0] == 1.0
    e[4] = float("inf")
    sgq.cluster_energy(plan, e, torch.tensor([0, 3, 5], device="cuda"),
                       torch.tensor([0, 1, 2, 3, 4], dtype=torch.int32, device="cuda"), None,
                       fbar[:2])
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_ENONFINITE
    # a good call clears the latch
    sgq.cluster_energy(plan, torch.arange(10, dtype=torch.float64, device="cuda"),
                       torch.tensor([0, 3, 5], device="cuda"),
                       torch.tensor([0, 1, 2, 3, 4], dtype=torch.int32, device="cuda"), None,
                       fbar[:2])
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    assert fbar[:2].cpu().numpy().tolist() == [1.0, 3.5]
    plan.close()


def test_cluster_energy_at_full_size_on_sampled_clusters():
    """The measured workload: 256 ESPs of the 64^3 system, 33-point balls (radius 1 bohr),
    autotuned launch.  Every Fbar_q is the mean of the device's own node energies (FP64
    rounding), the total equals the node-weighted band energy, and two sampled clusters
    are recomputed by the oracle node by node."""
    import torch
    from paper_1907_02604_amd import sgq
    P = synth.make_problem(2)
    esp = np.arange(256)
    Pn, cl = sgq.cluster_problem(P, esp, 1.0)
    plan = sgq.Plan.from_problem(Pn)
    v, R, E, wn = sgq.device_inputs(Pn)
    announce(f"cluster energy, full size: {Pn.n_nodes} merged nodes, autotuning")
    plan.autotune(v, R, E, Pn.mu, Pn.kT, sample_nodes=1024)
    e = torch.empty(Pn.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    sgq.band_energy(plan, v, R, E, wn, Pn.mu, Pn.kT, sgq.SGQ_FREE, e, om)
    off = torch.as_tensor(cl["member_offset"], device="cuda")
    mem = torch.as_tensor(cl["member_node"], device="cuda")
    we = torch.as_tensor(cl["esp_weight"], device="cuda")
    fbar = torch.empty(esp.size, dtype=torch.float64, device="cuda")
    en = torch.empty(1, dtype=torch.float64, device="cuda")
    sgq.cluster_energy(plan, e, off, mem, we, fbar, en)
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    e_h, f = e.cpu().numpy(), fbar.cpu().numpy()
    o, m = cl["member_offset"], cl["member_node"]
    means = np.array([e_h[m[a:b]].mean() for a, b in zip(o[:-1], o[1:])])
    assert np.max(np.abs(f - means)) <= 1e-13 * np.max(np.abs(e_h))
    assert abs(en.item() - om.item()) <= 1e-12 * abs(om.item())
    lookup = {int(p): i for i, p in enumerate(Pn.centers)}
    for q in (17, 200):
        members = O.cluster_members(P.n, P.h, int(P.centers[q]), 1.0)
        assert members.size == 33
        idx = [lookup[int(p)] for p in members]
        announce(f"cluster energy, full size: oracle on cluster {q}")
        ref_e, _ = O.band_energy(Pn, kind=O.FREE, nodes=idx)
        print("cluster", q, "fbar", f[q], "oracle", ref_e.mean())
        assert O.normwise_rel_err(e_h[idx], ref_e) < 1e-4
        assert abs(f[q] - ref_e.mean()) <= 1e-4 * np.max(np.abs(ref_e))
    plan.close()
