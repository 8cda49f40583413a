"""Benchmark: density nodes/s of the batched Lanczos-Gauss path on one MI355X.

Workload: 64^3 periodic grid (h = 0.5 bohr) with a jittered hcp Gaussian local
potential and four Kleinman-Bylander projectors per atom (255 atoms), 8192 seeded
nodes, 33^3 truncation cubes, Lanczos depth 60, FP32 matvecs with FP64 dots,
tridiagonal and quadrature.  One step = one rho_quadrature call over all nodes
(potential/projector setup kernels + the persistent Lanczos launch), inputs resident
in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-plain]
                    [--plain-nodes N] [--adjoint-nodes N]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "density nodes/sec and % HBM roofline at ≤1e-4 rel err, batched vs plain"
HBM_PEAK_GBS = 8000.0
KERNEL_SOURCES = ("sgq_common.h", "tridiag.h", "lanczos_device.h", "forward.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_lanczos_forward_64grid_8192nodes.txt")


def kernel_source_digest():
    """sha256 of the sources the forward kernel is built from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1907_02604_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or None when the
    kernel sources changed since the counters were taken."""
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != kernel_source_digest():
            return None
        return float(kv["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


def alg_bytes(n, K, elem=4):
    """Algorithmic bytes of one node: per step read q_j, q_{j-1}, write q_{j+1} and read
    the j earlier basis vectors once: elem * n * (3K + K(K+1)/2)."""
    return elem * n * (3 * K + K * (K + 1) / 2)


# ------------------------------------------------------------------ CPU baseline (oracle)
def _oracle_node(args):
    cfg, q = args
    import oracle as O
    from paper_1907_02604_amd import synth
    if "blas" not in _CACHE:
        # one BLAS thread per worker process: the pool already uses every core
        from threadpoolctl import threadpool_limits
        _CACHE["blas"] = threadpool_limits(1)
    P = _CACHE.get(cfg)
    if P is None:
        P = synth.make_problem(cfg)
        _CACHE[cfg] = P
    return O.rho_quadrature(P, nodes=[q])[0][0]


_CACHE = {}


def cpu_baseline(cfg, n_nodes_total, target_s=15.0):
    """Time the FP64 oracle on a seeded node sample, one process per core, before the
    GPU is touched: one untimed round lets every worker build the inputs, then rounds of
    one node per worker run until target_s has passed.  Returns (record, sample node ids,
    oracle rho of the sample)."""
    cores = min(16, os.cpu_count() or 1)
    rng = np.random.default_rng(1234)
    order = rng.permutation(n_nodes_total)
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        first = pool.map(_oracle_node, [(cfg, int(q)) for q in order[:cores]])
        done = cores
        timed = []
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < target_s and done + cores <= n_nodes_total:
            timed += pool.map(_oracle_node, [(cfg, int(q)) for q in order[done:done + cores]])
            done += cores
        wall = time.perf_counter() - t0
    n_timed = len(timed)
    rec = {"value": n_timed / wall, "unit": "nodes/s", "cores": cores, "kind": "oracle",
           "sample": f"{n_timed} seeded nodes of the 8192-node workload timed after a warm-up "
                     f"round of {cores}, FP64 numpy oracle, {cores} processes x 1 thread, "
                     f"{wall:.1f} s wall"}
    return rec, order[:done], np.array(first + timed)


# ------------------------------------------------------------------ GPU
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--plain-nodes", type=int, default=32)
    ap.add_argument("--adjoint-nodes", type=int, default=8192)
    ap.add_argument("--retain-gb", type=float, default=160.0,
                    help="retention budget of the dislocation sample's checkpointed adjoint "
                         "(GB of HBM for the Lanczos bases of its costliest nodes; 0: skip)")
    ap.add_argument("--dislocation-nodes", type=int, default=8192,
                    help="nodes of the dislocation-shaped sample (128^3 screw lattice, K=80): "
                         "forward and adjoint; 0 skips it")
    ap.add_argument("--cluster-esps", type=int, default=256,
                    help="energy sampling points of the cluster-energy leg (0 skips it)")
    ap.add_argument("--no-fe", action="store_true",
                    help="skip the fine-grid predictor + corrector reconstruction leg")
    ap.add_argument("--no-uneven", action="store_true",
                    help="skip the uneven-batching measurement (96^3, 20000 nodes, R and K drawn)")
    ap.add_argument("--tune-nodes", type=int, default=2048,
                    help="nodes of the sample the launch-shape autotuner times")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device-to-device copy first (reference for byte counters)")
    ap.add_argument("--config", type=int, default=2, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the node set would be dealt out by cost, one share per GPU).",
              file=sys.stderr)
        sys.exit(2)

    from paper_1907_02604_amd import synth
    cfg = args.config
    P = synth.make_problem(cfg)
    cpu_rec, sample, ref = (None, None, None)
    if not args.no_cpu:
        cpu_rec, sample, ref = cpu_baseline(cfg, P.n_nodes)
        print(f"[bench] cpu baseline {cpu_rec['value']:.2f} nodes/s on {cpu_rec['cores']} cores",
              file=sys.stderr, flush=True)
        import oracle as O          # the oracle timed beside the next-work legs

    import torch
    from paper_1907_02604_amd import sgq
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    plan = sgq.Plan.from_problem(P)
    v, R, E, _ = sgq.device_inputs(P)
    rho = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    # a stream of its own (default priority): the launch sequence is captured into a HIP
    # graph on the first call and replayed afterwards
    stream = torch.cuda.Stream()
    torch.cuda.synchronize()
    lanes, wg_per_cu = plan.autotune(v, R, E, P.mu, P.kT, sample_nodes=args.tune_nodes,
                                     stream=stream.cuda_stream)
    print(f"[bench] autotuned launch: {lanes} lanes per node, {wg_per_cu} workgroups per CU",
          file=sys.stderr, flush=True)

    def step():
        sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho, stream=stream.cuda_stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert plan.status() == sgq.SGQ_OK
    print(f"[bench] warmup done", file=sys.stderr, flush=True)
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        starts[i].record(stream)
        step()
        ends[i].record(stream)
    stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = [s.elapsed_time(e) for s, e in zip(starts, ends)]
    ms_per_step = wall * 1e3 / args.steps
    value = P.n_nodes * args.steps / wall
    assert plan.status() == sgq.SGQ_OK

    n_cube = int((2 * P.half_width[0] + 1) ** 3)
    K = int(P.depth[0])
    bytes_launch = float(sum(alg_bytes((2 * r + 1) ** 3, k) for r, k in zip(P.half_width, P.depth)))
    t_launch = float(np.mean(launch_ms)) * 1e-3
    achieved = bytes_launch / t_launch / 1e9
    traffic = measured_traffic()
    rec = {
        "metric": METRIC, "value": value, "unit": "nodes/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (seeded jittered-hcp Gaussian potential, U[-1,1] projector energies)",
        "config": {"workload": "64^3 grid h=0.5, 255 atoms with 4 KB projectors, 8192 nodes, "
                               "33^3 cubes, K=60, kT=0.01, mu=-0.1, FP32 matvec / FP64 dots",
                   "grid": list(P.n), "nodes": P.n_nodes, "cube_points": n_cube, "depth": K,
                   "launch": {"lanes_per_node": lanes, "workgroups_per_cu": wg_per_cu,
                              "autotuned": True, "hip_graph": True}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": f"lanczos_forward_kernel<float,{lanes},16>",
                     "alg_bytes_per_launch": bytes_launch, "avg_launch_ms": t_launch * 1e3,
                     # the sweep skips the leading basis rows of a block while they are still
                     # exactly zero there, so the HBM bytes it moves fall below the dense
                     # count above; this is the fraction of the peak those bytes make
                     "frac_of_measured_traffic": (traffic / t_launch / 1e9 / HBM_PEAK_GBS
                                                  if traffic else None)},
    }
    # Fermi level from the stored Gauss rules (no new Lanczos run): the count of the
    # density at mu = -0.1 is solved for its level again
    tw = torch.zeros(P.n_nodes * plan.kmax * 2, dtype=torch.float64, device="cuda")
    rho_f = torch.empty_like(rho)
    sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, rho_f, tw, stream=stream.cuda_stream)
    stream.synchronize()
    wq = torch.as_tensor(P.weight, dtype=torch.float64, device="cuda")
    n_el = float((rho_f * wq).sum().item()) * P.h ** 3
    fres = torch.empty(3, dtype=torch.float64, device="cuda")
    sgq.fermi_level(plan, tw, wq, n_el, P.kT, fres, stream=stream.cuda_stream)   # warm-up
    f0 = torch.cuda.Event(enable_timing=True)
    f1 = torch.cuda.Event(enable_timing=True)
    f0.record(stream)
    sgq.fermi_level(plan, tw, wq, n_el, P.kT, fres, stream=stream.cuda_stream)
    f1.record(stream)
    stream.synchronize()
    assert plan.status() == sgq.SGQ_OK
    fr = fres.cpu().numpy()
    rec["fermi_level"] = {"n_electrons": n_el, "mu": float(fr[0]), "mu_of_the_count": P.mu,
                          "steps": int(fr[2]), "ms": f0.elapsed_time(f1),
                          "rule_points": int(P.n_nodes * plan.kmax)}
    oracle_rows = {}
    if cpu_rec is not None:
        cpu_rec["next_rows"] = oracle_rows
        # the oracle's Brent solve on the same rules, on the host
        twh = tw.cpu().numpy().reshape(P.n_nodes, plan.kmax, 2)
        t0 = time.perf_counter()
        mu_o = O.fermi_level(twh[:, :, 0], twh[:, :, 1], P.weight, n_el, P.kT)
        oracle_rows["fermi_level"] = {"ms": (time.perf_counter() - t0) * 1e3,
                                      "mu_diff": abs(mu_o - float(fr[0])),
                                      "sample": "the same 491520 rule points, 1 thread"}
    if args.cluster_esps > 0:
        # cluster-sampled energy: balls of radius 1 bohr (33 grid points) around C2 nodes
        # taken as energy sampling points; the band energy of the merged ball nodes, then
        # the per-cluster means and the weighted total
        Pc, cl = sgq.cluster_problem(P, np.arange(args.cluster_esps), 1.0)
        cplan = sgq.Plan.from_problem(Pc)
        cplan.set_graph(True)
        cplan.autotune(v, R, E, Pc.mu, Pc.kT, sample_nodes=args.tune_nodes, stream=stream.cuda_stream)
        wn = torch.as_tensor(Pc.weight, device="cuda")
        ec = torch.empty(Pc.n_nodes, dtype=torch.float64, device="cuda")
        omc = torch.empty(1, dtype=torch.float64, device="cuda")
        off = torch.as_tensor(cl["member_offset"], device="cuda")
        mem = torch.as_tensor(cl["member_node"], device="cuda")
        we = torch.as_tensor(cl["esp_weight"], device="cuda")
        fbar = torch.empty(args.cluster_esps, dtype=torch.float64, device="cuda")
        en = torch.empty(1, dtype=torch.float64, device="cuda")

        def cluster_pass():
            sgq.band_energy(cplan, v, R, E, wn, Pc.mu, Pc.kT, sgq.SGQ_FREE, ec, omc,
                            stream=stream.cuda_stream)
            sgq.cluster_energy(cplan, ec, off, mem, we, fbar, en, stream=stream.cuda_stream)

        cluster_pass()                                   # warm-up (and graph capture)
        stream.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c2 = torch.cuda.Event(enable_timing=True)
        c0.record(stream)
        cluster_pass()
        c1.record(stream)
        sgq.cluster_energy(cplan, ec, off, mem, we, fbar, en, stream=stream.cuda_stream)
        c2.record(stream)
        stream.synchronize()
        assert cplan.status() == sgq.SGQ_OK
        tc = c0.elapsed_time(c1) * 1e-3
        rec["cluster_energy"] = {
            "workload": f"{args.cluster_esps} ESPs of the 64^3 system, balls of radius 1 bohr "
                        f"(33 points), {Pc.n_nodes} merged nodes, 33^3 cubes, K=60, FP32",
            "value": args.cluster_esps / tc, "unit": "ESPs/s", "nodes_per_s": Pc.n_nodes / tc,
            "pass_ms": tc * 1e3, "segmented_mean_ms": c1.elapsed_time(c2),
            "energy": en.item(), "omega_with_cluster_weights": omc.item()}
        print(f"[bench] cluster energy {args.cluster_esps / tc:.1f} ESPs/s "
              f"({Pc.n_nodes / tc:.1f} nodes/s)", file=sys.stderr, flush=True)
        cplan.close()
    if not args.no_fe:
        # predictor + corrector reconstruction of two fields (density, potential) on the
        # 128^3 fine grid from the ESPs of a coarse-grained dislocation run: the cylinder of
        # radius 4 points around the core line plus 65536 seeded points, Delaunay mesh
        n5 = (128, 128, 128)
        esp5 = synth.coarse_esps(n5, 5, 65536, 4)
        tets5 = synth.esp_mesh(n5, esp5)
        pred5 = synth.predictor_fields(n5, 0.5, synth.hcp_sites((64.0, 64.0, 64.0))).reshape(2, -1)
        ex, ey = esp5 % 128 - 64, (esp5 // 128) % 128 - 64
        decay = np.exp(-np.sqrt(ex * ex + ey * ey) / 6.0)
        vals5 = pred5[:, esp5] + np.stack([0.02 * decay, -0.3 * decay])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mesh = sgq.FeMesh(n5, esp5, tets5, max_fields=2)
        t_mesh = time.perf_counter() - t0
        pd = torch.as_tensor(np.ascontiguousarray(pred5), device="cuda")
        vd = torch.as_tensor(np.ascontiguousarray(vals5), device="cuda")
        od = torch.empty_like(pd)
        mesh.reconstruct(vd, pd, od, stream=stream.cuda_stream)       # warm-up
        stream.synchronize()
        reps = 50
        f0 = torch.cuda.Event(enable_timing=True)
        f1 = torch.cuda.Event(enable_timing=True)
        f0.record(stream)
        for _ in range(reps):
            mesh.reconstruct(vd, pd, od, stream=stream.cuda_stream)
        f1.record(stream)
        stream.synchronize()
        t_fe = f0.elapsed_time(f1) * 1e-3 / reps
        npts5 = 128 ** 3
        fe_bytes = npts5 * (4 + 2 * 16) + esp5.size * 2 * 24
        info = mesh.info()
        rec["fe_reconstruct"] = {
            "workload": f"128^3 fine grid, {esp5.size} ESPs (radius-4 core cylinder + 65536 "
                        f"seeded points), {info['kept']} Delaunay tetrahedra, 2 fields (rho, phi)",
            "value": npts5 / t_fe, "unit": "fine points/s", "us_per_call": t_fe * 1e6,
            "alg_bytes_per_call": fe_bytes, "achieved_GBs": fe_bytes / t_fe / 1e9,
            "frac_hbm_peak": fe_bytes / t_fe / 1e9 / HBM_PEAK_GBS,
            "mesh_create_s": t_mesh, "location_bucket": info["bucket"]}
        print(f"[bench] fe reconstruct {t_fe * 1e6:.1f} us/call, "
              f"{fe_bytes / t_fe / 1e9:.0f} GB/s; mesh + location {t_mesh:.2f} s",
              file=sys.stderr, flush=True)
        mesh.close()
        if cpu_rec is not None:
            # the oracle's brute-force location and 4x4 solves on 100 sampled fine points
            pts = np.random.default_rng(21).choice(npts5, 100, replace=False)
            t0 = time.perf_counter()
            ref_fe = O.fe_reconstruct(n5, esp5, tets5, vals5, pred5, points=pts)
            t_o = time.perf_counter() - t0
            err_fe = float(np.max(np.abs(od[:, pts].cpu().numpy() - ref_fe)) / np.max(np.abs(ref_fe)))
            oracle_rows["fe_reconstruct"] = {"value": 100 / t_o, "unit": "fine points/s",
                                             "max_rel_err_of_gpu": err_fe,
                                             "sample": "100 seeded fine points, 1 thread"}
        # the potential of the next self-consistency step from the reconstructed density:
        # V = phi[rho + b] + u(rho) on the same 128^3 grid (periodic FFT Poisson solve with the
        # FD Laplacian, LDA exchange-correlation fused into its last pass)
        bq = torch.as_tensor(synth.nuclear_charge(n5, 0.5, synth.hcp_sites((64.0, 64.0, 64.0))),
                             device="cuda").reshape(-1)
        rho5 = od[0].clamp(min=0.0).contiguous()
        pot = sgq.Potential(n5, 0.5)
        vpot = torch.empty_like(rho5)
        pot.effective(rho5, vpot, b=bq, stream=stream.cuda_stream)    # warm-up
        stream.synchronize()
        f0.record(stream)
        for _ in range(reps):
            pot.effective(rho5, vpot, b=bq, stream=stream.cuda_stream)
        f1.record(stream)
        stream.synchronize()
        t_pot = f0.elapsed_time(f1) * 1e-3 / reps
        # five line passes over the half-spectrum complex grid (65 x 128 x 128, 16 B each): X
        # forward reads rho and b and writes the grid, the Y, Z (solve) and Y inverse passes
        # read and write it, the X inverse pass reads it and rho and writes V
        cpts5 = (128 // 2 + 1) * 128 * 128
        pot_bytes = npts5 * 32 + cpts5 * 16 * 8
        rec["effective_potential"] = {
            "workload": "128^3 grid, V = phi[rho + b] + u_xc(rho) from the reconstructed density "
                        "and Gaussian nuclear charges (Z = 2) at the lattice sites, FP64",
            "value": npts5 / t_pot, "unit": "grid points/s", "us_per_call": t_pot * 1e6,
            "bytes_per_call": pot_bytes, "achieved_GBs": pot_bytes / t_pot / 1e9,
            "frac_hbm_peak": pot_bytes / t_pot / 1e9 / HBM_PEAK_GBS}
        print(f"[bench] effective potential {t_pot * 1e6:.1f} us/call, "
              f"{pot_bytes / t_pot / 1e9:.0f} GB/s", file=sys.stderr, flush=True)
        if cpu_rec is not None:
            t0 = time.perf_counter()
            ref_v, _, _, _ = O.effective_potential(rho5.cpu().numpy().reshape(128, 128, 128),
                                                   bq.cpu().numpy().reshape(128, 128, 128), 0.5)
            t_o = time.perf_counter() - t0
            got_v = vpot.cpu().numpy().reshape(128, 128, 128)
            oracle_rows["effective_potential"] = {
                "value": npts5 / t_o, "unit": "grid points/s",
                "max_rel_err_of_gpu": float(np.max(np.abs(got_v - ref_v)) / np.max(np.abs(ref_v))),
                "sample": "the whole 128^3 grid, numpy FFT"}
        pot.close()
    if not args.no_plain:
        # per-node GPU baseline: the plain schedule on a seeded node sample
        idx = np.random.default_rng(7).choice(P.n_nodes, args.plain_nodes, replace=False)
        Q = P.subset(np.sort(idx))
        pplan = sgq.Plan.from_problem(Q)
        pplan.set_schedule(sgq.SGQ_SCHEDULE_PLAIN)
        prho = torch.empty(Q.n_nodes, dtype=torch.float64, device="cuda")
        sgq.rho_quadrature(pplan, v, R, E, Q.mu, Q.kT, prho)       # warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sgq.rho_quadrature(pplan, v, R, E, Q.mu, Q.kT, prho)
        torch.cuda.synchronize()
        tp = time.perf_counter() - t0
        assert pplan.status() == sgq.SGQ_OK
        perr = float(np.max(np.abs(prho.cpu().numpy() - rho.cpu().numpy()[np.sort(idx)]))
                     / np.max(np.abs(rho.cpu().numpy()[np.sort(idx)])))
        rec["plain"] = {"value": Q.n_nodes / tp, "unit": "nodes/s", "nodes": Q.n_nodes,
                        "schedule": "one node at a time, grid-wide kernels per Lanczos step",
                        "rel_diff_vs_batched": perr,
                        "batched_speedup": value / (Q.n_nodes / tp)}
        pplan.close()
        print(f"[bench] plain {Q.n_nodes / tp:.1f} nodes/s", file=sys.stderr, flush=True)
    if args.adjoint_nodes > 0:
        # adjoint throughput on the differentiation workload (48^3, 16 atoms, 33^3 cubes,
        # K = 60): forward recompute + reverse recurrence + gathers, on a node sample
        P4 = synth.make_problem(4)
        idx = np.random.default_rng(8).choice(P4.n_nodes, args.adjoint_nodes, replace=False)
        Q4 = P4.subset(np.sort(idx))
        aplan = sgq.Plan.from_problem(Q4)
        v4, R4, E4, w4 = sgq.device_inputs(Q4)
        g = torch.ones(1, dtype=torch.float64, device="cuda")
        dV = torch.empty_like(v4)
        dR = torch.zeros_like(R4)
        dE = torch.zeros_like(E4)
        sgq.band_energy_backward(aplan, v4, R4, E4, w4, Q4.mu, Q4.kT, sgq.SGQ_FREE, g, dV, dR, dE)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sgq.band_energy_backward(aplan, v4, R4, E4, w4, Q4.mu, Q4.kT, sgq.SGQ_FREE, g, dV, dR, dE)
        torch.cuda.synchronize()
        ta = time.perf_counter() - t0
        assert aplan.status() == sgq.SGQ_OK
        # algorithmic bytes of one node's adjoint: the forward recompute B(n, K), the adjoint
        # vectors and their matvec 4n*8K, the node's dV cube 4n
        abytes = float(sum(alg_bytes((2 * r + 1) ** 3, k) + 4.0 * (2 * r + 1) ** 3 * (8 * k + 1)
                           for r, k in zip(Q4.half_width, Q4.depth)))
        rec["adjoint"] = {"value": Q4.n_nodes / ta, "unit": "nodes/s", "nodes": Q4.n_nodes,
                          "workload": "48^3 grid, 16 atoms with KB projectors, 33^3 cubes, K=60, "
                                      "FP32, dOmega/dV + dOmega/dR + dOmega/dE",
                          "alg_bytes": abytes, "achieved_GBs": abytes / ta / 1e9,
                          "frac_hbm_peak": abytes / ta / 1e9 / HBM_PEAK_GBS}
        print(f"[bench] adjoint {Q4.n_nodes / ta:.1f} nodes/s", file=sys.stderr, flush=True)
        # the same adjoint after a forward call that retained its bases (per-node storage of
        # the Lanczos vectors and u_j rows, 141 GB here), so the backward skips the recompute
        dV_re = dV.clone()
        aplan.set_retain(True)
        e4 = torch.empty(Q4.n_nodes, dtype=torch.float64, device="cuda")
        om4 = torch.empty(1, dtype=torch.float64, device="cuda")
        sgq.band_energy(aplan, v4, R4, E4, w4, Q4.mu, Q4.kT, sgq.SGQ_FREE, e4, om4)   # warm-up
        sgq.band_energy_backward(aplan, v4, R4, E4, w4, Q4.mu, Q4.kT, sgq.SGQ_FREE, g, dV, dR, dE)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sgq.band_energy(aplan, v4, R4, E4, w4, Q4.mu, Q4.kT, sgq.SGQ_FREE, e4, om4)
        torch.cuda.synchronize()
        tf = time.perf_counter() - t0
        t0 = time.perf_counter()
        sgq.band_energy_backward(aplan, v4, R4, E4, w4, Q4.mu, Q4.kT, sgq.SGQ_FREE, g, dV, dR, dE)
        torch.cuda.synchronize()
        tb = time.perf_counter() - t0
        assert aplan.status() == sgq.SGQ_OK
        rec["adjoint"]["retained_bases"] = {
            "value": Q4.n_nodes / tb, "unit": "nodes/s", "forward_s": tf, "backward_s": tb,
            "forward_plus_backward_nodes_per_s": Q4.n_nodes / (tf + tb),
            "forward_plus_recompute_backward_nodes_per_s": Q4.n_nodes / (tf + ta),
            "dV_bitwise_equal_to_recompute": bool(torch.equal(dV, dV_re))}
        aplan.close()
        print(f"[bench] adjoint with retained bases {Q4.n_nodes / tb:.1f} nodes/s "
              f"(forward + backward {Q4.n_nodes / (tf + tb):.1f} nodes/s)", file=sys.stderr, flush=True)
    if not args.no_uneven:
        # uneven batching: 20000 nodes with radii U{6..12} bohr and depths U{40..100} in one
        # persistent, autotuned, graph-replayed launch
        P3 = synth.make_problem(3)
        uplan = sgq.Plan.from_problem(P3)
        v3, R3, E3, _ = sgq.device_inputs(P3)
        rho3 = torch.empty(P3.n_nodes, dtype=torch.float64, device="cuda")
        shape3 = uplan.autotune(v3, R3, E3, P3.mu, P3.kT, sample_nodes=args.tune_nodes,
                                stream=stream.cuda_stream)
        sgq.rho_quadrature(uplan, v3, R3, E3, P3.mu, P3.kT, rho3, stream=stream.cuda_stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sgq.rho_quadrature(uplan, v3, R3, E3, P3.mu, P3.kT, rho3, stream=stream.cuda_stream)
        e1.record(stream)
        stream.synchronize()
        t3 = e0.elapsed_time(e1) * 1e-3
        assert uplan.status() == sgq.SGQ_OK
        b3 = float(sum(alg_bytes((2 * r + 1) ** 3, k) for r, k in zip(P3.half_width, P3.depth)))
        costs = [alg_bytes((2 * r + 1) ** 3, k) for r, k in zip(P3.half_width, P3.depth)]
        rec["uneven"] = {"value": P3.n_nodes / t3, "unit": "nodes/s", "nodes": P3.n_nodes,
                         "workload": "96^3 grid h=0.5, 760 atoms with KB projectors, radii "
                                     "U{6..12} bohr (cubes 25^3..49^3), depths U{40..100}, "
                                     "kT=0.005, FP32",
                         "launch_ms": t3 * 1e3, "alg_bytes": b3, "achieved_GBs": b3 / t3 / 1e9,
                         "frac_hbm_peak": b3 / t3 / 1e9 / HBM_PEAK_GBS,
                         "node_cost_spread": max(costs) / min(costs),
                         "launch": {"lanes_per_node": shape3[0], "workgroups_per_cu": shape3[1],
                                    "autotuned": True, "hip_graph": True}}
        uplan.close()
        print(f"[bench] uneven {P3.n_nodes / t3:.1f} nodes/s", file=sys.stderr, flush=True)
    if args.dislocation_nodes > 0:
        # dislocation-shaped input: 128^3 screw-displaced lattice, radii 6..12 bohr, K = 80,
        # node weights 32; forward (autotuned, graph-replayed) and adjoint on a node sample
        P5 = synth.make_problem(5)
        Q5 = P5.subset(np.arange(min(args.dislocation_nodes, P5.n_nodes)))
        dplan = sgq.Plan.from_problem(Q5)
        v5, R5, E5, w5 = sgq.device_inputs(Q5)
        rho5 = torch.empty(Q5.n_nodes, dtype=torch.float64, device="cuda")
        shape5 = dplan.autotune(v5, R5, E5, Q5.mu, Q5.kT, sample_nodes=args.tune_nodes,
                                stream=stream.cuda_stream)
        sgq.rho_quadrature(dplan, v5, R5, E5, Q5.mu, Q5.kT, rho5, stream=stream.cuda_stream)
        stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        sgq.rho_quadrature(dplan, v5, R5, E5, Q5.mu, Q5.kT, rho5, stream=stream.cuda_stream)
        e1.record(stream)
        stream.synchronize()
        t5 = e0.elapsed_time(e1) * 1e-3
        assert dplan.status() == sgq.SGQ_OK
        b5 = float(sum(alg_bytes((2 * r + 1) ** 3, k) for r, k in zip(Q5.half_width, Q5.depth)))
        g5 = torch.ones(1, dtype=torch.float64, device="cuda")
        dV5 = torch.empty_like(v5)
        dR5 = torch.zeros_like(R5)
        dE5 = torch.zeros_like(E5)
        sgq.band_energy_backward(dplan, v5, R5, E5, w5, Q5.mu, Q5.kT, sgq.SGQ_FREE, g5, dV5, dR5, dE5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sgq.band_energy_backward(dplan, v5, R5, E5, w5, Q5.mu, Q5.kT, sgq.SGQ_FREE, g5, dV5, dR5, dE5)
        torch.cuda.synchronize()
        tb5 = time.perf_counter() - t0
        assert dplan.status() == sgq.SGQ_OK
        rec["dislocation"] = {
            "workload": f"128^3 grid h=0.5, 1925 screw-displaced atoms with KB projectors, "
                        f"{Q5.n_nodes} of 65536 nodes (weights 32), cubes 25^3..49^3, K=80, "
                        f"kT=0.005, FP32",
            "forward": {"value": Q5.n_nodes / t5, "unit": "nodes/s", "launch_ms": t5 * 1e3,
                        "achieved_GBs": b5 / t5 / 1e9, "frac_hbm_peak": b5 / t5 / 1e9 / HBM_PEAK_GBS,
                        "launch": {"lanes_per_node": shape5[0], "workgroups_per_cu": shape5[1]}},
            "adjoint": {"value": Q5.n_nodes / tb5, "unit": "nodes/s", "s": tb5}}
        if args.retain_gb > 0:
            # the adjoint with checkpointed Lanczos vectors: the forward keeps the bases and
            # u_j rows of the costliest nodes that fit in the budget, and the backward
            # recomputes only the others
            free_b, _ = torch.cuda.mem_get_info()
            budget = int(min(args.retain_gb * 1e9, free_b - 24e9))
            try:
                n_ret = dplan.set_retain(True, max_bytes=budget) if budget > 0 else 0
            except sgq.SgqError as err:
                n_ret = 0
                print(f"[bench] no checkpointed adjoint: {err}", file=sys.stderr, flush=True)
            if n_ret > 0:
                dV5_re = dV5.clone()
                e5 = torch.empty(Q5.n_nodes, dtype=torch.float64, device="cuda")
                om5 = torch.empty(1, dtype=torch.float64, device="cuda")
                sgq.band_energy(dplan, v5, R5, E5, w5, Q5.mu, Q5.kT, sgq.SGQ_FREE, e5, om5)
                sgq.band_energy_backward(dplan, v5, R5, E5, w5, Q5.mu, Q5.kT, sgq.SGQ_FREE, g5,
                                         dV5, dR5, dE5)   # warm-up pair
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                sgq.band_energy(dplan, v5, R5, E5, w5, Q5.mu, Q5.kT, sgq.SGQ_FREE, e5, om5)
                torch.cuda.synchronize()
                tf5 = time.perf_counter() - t0
                t0 = time.perf_counter()
                sgq.band_energy_backward(dplan, v5, R5, E5, w5, Q5.mu, Q5.kT, sgq.SGQ_FREE, g5,
                                         dV5, dR5, dE5)
                torch.cuda.synchronize()
                tc5 = time.perf_counter() - t0
                assert dplan.status() == sgq.SGQ_OK
                rec["dislocation"]["adjoint"]["checkpointed"] = {
                    "value": Q5.n_nodes / tc5, "unit": "nodes/s", "s": tc5,
                    "retained_nodes": n_ret, "budget_GB": budget / 1e9,
                    "forward_s": tf5, "forward_plus_backward_nodes_per_s": Q5.n_nodes / (tf5 + tc5),
                    "forward_plus_recompute_backward_nodes_per_s": Q5.n_nodes / (t5 + tb5),
                    # the forward ran with the autotuned lanes per node, the recompute with
                    # the backward's 256: the two gradients differ by FP32 rounding only
                    "dV_normwise_rel_diff_vs_recompute":
                        float((dV5 - dV5_re).abs().max() / dV5_re.abs().max())}
                print(f"[bench] dislocation checkpointed adjoint {Q5.n_nodes / tc5:.1f} nodes/s "
                      f"({n_ret} of {Q5.n_nodes} nodes retained)", file=sys.stderr, flush=True)
            dplan.set_retain(False)
        dplan.close()
        print(f"[bench] dislocation fwd {Q5.n_nodes / t5:.1f} adj {Q5.n_nodes / tb5:.1f} nodes/s",
              file=sys.stderr, flush=True)
    if cpu_rec is not None:
        got = rho.cpu().numpy()[sample]
        err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
        rec["cpu_baseline"] = cpu_rec
        rec["accuracy"] = {"normwise_rel_err_vs_fp64_oracle": err, "nodes_checked": int(len(sample))}
    print(json.dumps(rec), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
