"""Benchmark: density nodes/s of the batched Lanczos-Gauss path on one MI355X.

Headline workload: 64^3 periodic grid (h = 0.5 bohr) with a jittered hcp Gaussian local
potential and four Kleinman-Bylander projectors per atom (255 atoms), 8192 seeded nodes,
33^3 truncation cubes, Lanczos depth 60, FP32 matvecs with FP64 dots, tridiagonal and
quadrature.  One step = one rho_quadrature call over all nodes (potential/projector setup
kernels + the persistent Lanczos launch), inputs resident in HBM.

The other workloads are measured once each at their full sizes: the 16^3 untruncated FP64
grid (all 4096 points), the 96^3 uneven batch (20000 nodes), the 48^3 differentiation
workload (all 110592 nodes, forward and adjoint) and the 128^3 dislocation-shaped workload
(all 65536 nodes, forward, adjoint and the adjoint with checkpointed Lanczos vectors).
Before the GPU is touched, the FP64 oracle is timed on seeded samples of every workload
(stratified by node cost), on all the host cores the box grants and on one thread; the
same samples give each GPU result's error against the oracle.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--legs a,b,...]
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
LEGS = ("copy", "fermi", "cluster", "fe", "plain", "c1", "c3", "c4", "c5")
# host cores granted to a job per GPU on the target nodes, whatever nproc reports
HOST_CORE_SHARE = 16


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


def cube_points(half_width, n_grid):
    """Points of each node's cube (the whole grid for an untruncated node)."""
    hw = np.asarray(half_width, dtype=np.int64)
    return np.where(hw < 0, int(np.prod(n_grid)), (2 * hw + 1) ** 3)


def launch_bytes(prob, elem=4):
    n = cube_points(prob.half_width, prob.n)
    return float(sum(alg_bytes(int(a), int(k), elem) for a, k in zip(n, prob.depth)))


def stratified_order(cost, n_bins, seed):
    """Node ids in an order whose every run of n_bins consecutive entries holds one node of
    each cost stratum (nodes sorted by cost and split into n_bins equal bins), each bin
    visited in a seeded random order: any prefix is a stratified sample."""
    order = np.argsort(np.asarray(cost), kind="stable")
    bins = [np.random.default_rng(seed + i).permutation(b)
            for i, b in enumerate(np.array_split(order, n_bins)) if b.size]
    out = []
    for r in range(max(b.size for b in bins)):
        out += [int(b[r]) for b in bins if r < b.size]
    return np.array(out, dtype=np.int64)


def node_cost(prob):
    n = cube_points(prob.half_width, prob.n).astype(np.float64)
    K = prob.depth.astype(np.float64)
    return n * (3 * K + K * (K + 1) / 2)


def errors(got, ref, floor=1e-3):
    """Normwise ||got - ref||_inf / ||ref||_inf and the largest per-node relative error over
    the nodes with |ref| > floor * ||ref||_inf."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    den = float(np.max(np.abs(ref)))
    sig = np.abs(ref) > floor * den
    return {"normwise_rel_err": float(np.max(np.abs(got - ref)) / den),
            "per_node_rel_err_max": float(np.max(np.abs(got[sig] - ref[sig]) / np.abs(ref[sig]))),
            "per_node_floor": floor, "nodes_checked": int(ref.size),
            "nodes_above_floor": int(sig.sum())}


# ------------------------------------------------------------------ CPU baseline (oracle)
_PROBLEMS = {}


def _oracle_node(args):
    cfg, q = args
    import oracle as O
    if "blas" not in _PROBLEMS:
        # one BLAS thread per worker process: the pool already uses every core it has
        from threadpoolctl import threadpool_limits
        _PROBLEMS["blas"] = threadpool_limits(1)
    return float(O.rho_quadrature(_PROBLEMS[cfg], nodes=[q])[0][0])


def cpu_baselines(cfgs, target_s, target_1t):
    """Time the FP64 oracle on a stratified seeded node sample of every workload, before the
    GPU is touched: a pool of one process per granted core (one untimed warm-up round, then
    rounds of one node per process until target_s[cfg] has passed), then one thread in this
    process on further nodes of the same order for target_1t seconds.  Returns
    {cfg: (record, node ids, oracle rho of those nodes)}."""
    from paper_1907_02604_amd import synth
    from threadpoolctl import threadpool_limits
    import oracle as O
    nproc = os.cpu_count() or 1
    try:
        granted = len(os.sched_getaffinity(0))
    except AttributeError:
        granted = nproc
    cores = max(1, min(HOST_CORE_SHARE, granted))
    orders = {}
    for cfg in cfgs:
        P = synth.make_problem(cfg)
        _PROBLEMS[cfg] = P          # built before the fork: the workers share it
        orders[cfg] = stratified_order(node_cost(P), min(64, P.n_nodes), 100 + cfg)
    out = {}
    ctx = mp.get_context("fork")
    with ctx.Pool(cores) as pool:
        for cfg in cfgs:
            order = orders[cfg]
            nq = order.size
            first = pool.map(_oracle_node, [(cfg, int(q)) for q in order[:cores]])
            done, timed = min(cores, nq), []
            t0 = time.perf_counter()
            while time.perf_counter() - t0 < target_s[cfg] and done < nq:
                chunk = order[done:done + cores]
                timed += pool.map(_oracle_node, [(cfg, int(q)) for q in chunk])
                done += chunk.size
            wall = time.perf_counter() - t0
            if not timed:     # the warm-up round took every node: time one more round
                t0 = time.perf_counter()
                pool.map(_oracle_node, [(cfg, int(q)) for q in order[:cores]])
                wall, n_rate = time.perf_counter() - t0, min(cores, nq)
            else:
                n_rate = len(timed)
            out[cfg] = {"ids": order[:done], "rho": np.array(first + timed),
                        "all": {"value": n_rate / wall, "nodes": n_rate, "wall_s": wall,
                                "processes": cores}}
    with threadpool_limits(1):
        for cfg in cfgs:
            # further nodes of the same order (from its start again once the pool has done
            # them all: then only the time counts)
            order, ids = orders[cfg], out[cfg]["ids"]
            start, n1 = ids.size, 0
            vals = []
            t0 = time.perf_counter()
            while n1 == 0 or time.perf_counter() - t0 < target_1t[cfg]:
                k = (start + n1) % order.size
                r = float(O.rho_quadrature(_PROBLEMS[cfg], nodes=[int(order[k])])[0][0])
                if start + n1 < order.size:
                    vals.append(r)
                n1 += 1
            wall = time.perf_counter() - t0
            out[cfg]["one"] = {"value": n1 / wall, "nodes": n1, "wall_s": wall}
            out[cfg]["ids"] = order[:start + len(vals)]
            out[cfg]["rho"] = np.concatenate([out[cfg]["rho"], vals])
    for cfg in cfgs:
        out[cfg]["nproc"], out[cfg]["granted"] = nproc, granted
    return out


def cpu_record(base, cfg, desc):
    a, o = base[cfg]["all"], base[cfg]["one"]
    return {"value": a["value"], "unit": "nodes/s", "cores": a["processes"], "kind": "oracle",
            "nproc": base[cfg]["nproc"], "cores_granted": base[cfg]["granted"],
            "one_thread": {"value": o["value"], "nodes": o["nodes"], "wall_s": o["wall_s"]},
            "sample": f"{a['nodes']} nodes of {desc} (stratified by cost, seeded) after a warm-up "
                      f"round, FP64 numpy oracle, {a['processes']} processes x 1 BLAS thread, "
                      f"{a['wall_s']:.1f} s wall; one thread: {o['nodes']} more nodes, "
                      f"{o['wall_s']:.1f} s"}


# ------------------------------------------------------------------ GPU helpers
def event_time(stream, fn):
    """Seconds between HIP events recorded on `stream` around fn()."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    fn()
    e1.record(stream)
    stream.synchronize()
    return e0.elapsed_time(e1) * 1e-3


def copy_peak():
    """Device-to-device copy of 1 GiB (read 1 GiB, write 1 GiB) and a 4 GiB streaming read
    (a reduction), best of five, as GB/s of bytes moved."""
    import torch
    src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    big = torch.ones(1 << 30, dtype=torch.float32, device="cuda")
    s = torch.cuda.current_stream()
    dst.copy_(src)
    big.sum()
    torch.cuda.synchronize()
    tc = min(event_time(s, lambda: dst.copy_(src)) for _ in range(5))
    tr = min(event_time(s, lambda: big.sum()) for _ in range(5))
    rec = {"copy_GBs": 2.0 * src.numel() * 4 / tc / 1e9, "copy_bytes": 2 * src.numel() * 4,
           "read_GBs": big.numel() * 4 / tr / 1e9, "read_bytes": big.numel() * 4,
           "method": "torch copy_ of 1 GiB device to device (hipMemcpy kernel) and torch sum of "
                     "4 GiB of FP32, HIP events, best of 5"}
    del src, dst, big
    torch.cuda.empty_cache()
    return rec


def forward_leg(sgq, torch, P, stream, tune_nodes, kind=None, warm=False):
    """Plan, autotune and one timed forward launch of problem P (density, or the energy
    with kind).  With warm, an untimed call first captures the launch graph and the timed
    call replays it; without, the timed call launches directly (a multi-second launch needs
    no warm-up).  Returns (plan, rho or e_node tensor, seconds, launch shape, inputs,
    omega)."""
    plan = sgq.Plan.from_problem(P)
    if not warm:
        plan.set_graph(False)
    v, R, E, w = sgq.device_inputs(P)
    out = torch.empty(P.n_nodes, dtype=torch.float64, device="cuda")
    om = torch.empty(1, dtype=torch.float64, device="cuda")
    shape = plan.autotune(v, R, E, P.mu, P.kT, sample_nodes=tune_nodes, stream=stream.cuda_stream)

    def run():
        if kind is None:
            sgq.rho_quadrature(plan, v, R, E, P.mu, P.kT, out, stream=stream.cuda_stream)
        else:
            sgq.band_energy(plan, v, R, E, w, P.mu, P.kT, kind, out, om, stream=stream.cuda_stream)

    if warm:
        run()
        stream.synchronize()
    t = event_time(stream, run)
    assert plan.status() == sgq.SGQ_OK
    return plan, out, t, shape, (v, R, E, w), om


def base_nodes(cfg):
    return {1: 4096, 2: 8192, 3: 20000, 4: 110592, 5: 65536}[cfg]


def accuracy(base, cfg, values):
    if base is None or cfg not in base:
        return None
    ids, ref = base[cfg]["ids"], base[cfg]["rho"]
    return errors(values[ids], ref)


# ------------------------------------------------------------------ main
def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated legs besides the headline: " + ",".join(LEGS))
    ap.add_argument("--plain-nodes", type=int, default=32)
    ap.add_argument("--retain-gb", type=float, default=160.0,
                    help="retention budget of the checkpointed adjoints (GB of HBM for the "
                         "Lanczos bases of the costliest nodes; 0: skip)")
    ap.add_argument("--cluster-esps", type=int, default=256)
    ap.add_argument("--adjoint-nodes", type=int, default=0,
                    help="run the differentiation leg on this many seeded nodes instead of all "
                         "110592 (0: all)")
    ap.add_argument("--tune-nodes", type=int, default=2048,
                    help="nodes of the sample the launch-shape autotuner times")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device-to-device copy first (reference for byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the node set would be dealt out by cost, one share per GPU).",
              file=sys.stderr)
        sys.exit(2)
    legs = set(x for x in args.legs.split(",") if x)
    unknown = legs - set(LEGS)
    if unknown:
        print(f"unknown legs: {sorted(unknown)}", file=sys.stderr)
        sys.exit(2)

    from paper_1907_02604_amd import synth
    P = synth.make_problem(2)
    base = None
    if not args.no_cpu:
        cfgs = [2] + [c for c, leg in ((1, "c1"), (3, "c3"), (4, "c4"), (5, "c5")) if leg in legs]
        target = {1: 3.0, 2: 10.0, 3: 8.0, 4: 5.0, 5: 8.0}
        target1 = {1: 2.0, 2: 4.0, 3: 4.0, 4: 3.0, 5: 4.0}
        base = cpu_baselines(cfgs, target, target1)
        for c in cfgs:
            print(f"[bench] oracle C{c}: {base[c]['all']['value']:.2f} nodes/s on "
                  f"{base[c]['all']['processes']} processes, {base[c]['one']['value']:.2f} on "
                  f"one thread", file=sys.stderr, flush=True)
        import oracle as O          # the oracle timed beside the next-work legs

    import torch
    from paper_1907_02604_amd import sgq
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    peak = copy_peak() if "copy" in legs else None
    if peak:
        print(f"[bench] copy {peak['copy_GBs']:.0f} GB/s, read {peak['read_GBs']:.0f} GB/s",
              file=sys.stderr, flush=True)

    # ---------------- headline: the 64^3 workload, K steps of one launch each
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
    print("[bench] warmup done", file=sys.stderr, flush=True)
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
    bytes_launch = launch_bytes(P)
    t_launch = float(np.mean(launch_ms)) * 1e-3
    achieved = bytes_launch / t_launch / 1e9
    traffic = measured_traffic()
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "kernel": f"lanczos_forward_kernel<float,{lanes},16>",
            "alg_bytes_per_launch": bytes_launch, "avg_launch_ms": t_launch * 1e3,
            # the sweep skips the leading basis rows of a block while they are still exactly
            # zero there, so the HBM bytes it moves fall below the dense count above; this is
            # the fraction of the peak those bytes make
            "frac_of_measured_traffic": (traffic / t_launch / 1e9 / HBM_PEAK_GBS
                                         if traffic else None)}
    if peak:
        roof["measured_copy_GBs"] = peak["copy_GBs"]
        roof["measured_read_GBs"] = peak["read_GBs"]
        roof["frac_of_measured_copy"] = achieved / peak["copy_GBs"]
        if traffic:
            roof["measured_traffic_frac_of_measured_copy"] = traffic / t_launch / 1e9 / peak["copy_GBs"]
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
        "roofline": roof,
    }
    if peak:
        rec["hbm_measured"] = peak
    rho_c2 = rho.cpu().numpy()
    oracle_rows = {}

    if "fermi" in legs:
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
        tf = event_time(stream, lambda: sgq.fermi_level(plan, tw, wq, n_el, P.kT, fres,
                                                        stream=stream.cuda_stream))
        assert plan.status() == sgq.SGQ_OK
        fr = fres.cpu().numpy()
        rec["fermi_level"] = {"n_electrons": n_el, "mu": float(fr[0]), "mu_of_the_count": P.mu,
                              "steps": int(fr[2]), "ms": tf * 1e3,
                              "rule_points": int(P.n_nodes * plan.kmax)}
        if base is not None:
            twh = tw.cpu().numpy().reshape(P.n_nodes, plan.kmax, 2)
            t0 = time.perf_counter()
            mu_o = O.fermi_level(twh[:, :, 0], twh[:, :, 1], P.weight, n_el, P.kT)
            oracle_rows["fermi_level"] = {"ms": (time.perf_counter() - t0) * 1e3,
                                          "mu_diff": abs(mu_o - float(fr[0])),
                                          "sample": "the same 491520 rule points, 1 thread"}
        del tw, rho_f
    if "cluster" in legs and args.cluster_esps > 0:
        # cluster-sampled energy: balls of radius 1 bohr (33 grid points) around C2 nodes
        # taken as energy sampling points; the band energy of the merged ball nodes, then
        # the per-cluster means and the weighted total
        Pc, cl = sgq.cluster_problem(P, np.arange(args.cluster_esps), 1.0)
        cplan = sgq.Plan.from_problem(Pc)
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
        tc = event_time(stream, cluster_pass)
        tm = event_time(stream, lambda: sgq.cluster_energy(cplan, ec, off, mem, we, fbar, en,
                                                           stream=stream.cuda_stream))
        assert cplan.status() == sgq.SGQ_OK
        rec["cluster_energy"] = {
            "workload": f"{args.cluster_esps} ESPs of the 64^3 system, balls of radius 1 bohr "
                        f"(33 points), {Pc.n_nodes} merged nodes, 33^3 cubes, K=60, FP32",
            "value": args.cluster_esps / tc, "unit": "ESPs/s", "nodes_per_s": Pc.n_nodes / tc,
            "pass_ms": tc * 1e3, "segmented_mean_ms": tm * 1e3,
            "energy": en.item(), "omega_with_cluster_weights": omc.item()}
        print(f"[bench] cluster energy {args.cluster_esps / tc:.1f} ESPs/s "
              f"({Pc.n_nodes / tc:.1f} nodes/s)", file=sys.stderr, flush=True)
        cplan.close()
    if "fe" in legs:
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

        def fe_reps():
            for _ in range(reps):
                mesh.reconstruct(vd, pd, od, stream=stream.cuda_stream)

        t_fe = event_time(stream, fe_reps) / reps
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
        if base is not None:
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

        def pot_reps():
            for _ in range(reps):
                pot.effective(rho5, vpot, b=bq, stream=stream.cuda_stream)

        t_pot = event_time(stream, pot_reps) / reps
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
        if base is not None:
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
        del pd, vd, od, bq, rho5, vpot
    if "plain" in legs:
        # per-node GPU baseline: the plain schedule on a seeded node sample
        idx = np.sort(np.random.default_rng(7).choice(P.n_nodes, args.plain_nodes, replace=False))
        Q = P.subset(idx)
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
        perr = float(np.max(np.abs(prho.cpu().numpy() - rho_c2[idx])) / np.max(np.abs(rho_c2[idx])))
        rec["plain"] = {"value": Q.n_nodes / tp, "unit": "nodes/s", "nodes": Q.n_nodes,
                        "schedule": "one node at a time, grid-wide kernels per Lanczos step",
                        "rel_diff_vs_batched": perr,
                        "batched_speedup": value / (Q.n_nodes / tp)}
        pplan.close()
        print(f"[bench] plain {Q.n_nodes / tp:.1f} nodes/s", file=sys.stderr, flush=True)
    plan.close()
    del v, R, E, rho
    torch.cuda.empty_cache()

    configs = {}
    if "c1" in legs:
        # untruncated FP64 path: every point of the 16^3 periodic grid, K = 30
        P1 = synth.make_problem(1)
        p1, rho1, t1, shape1, _, _ = forward_leg(sgq, torch, P1, stream, args.tune_nodes, warm=True)
        b1 = launch_bytes(P1, elem=8)
        configs["c1"] = {
            "workload": "16^3 periodic grid h=0.5, 6 atoms, no projectors, all 4096 points "
                        "untruncated (the whole periodic H), K=30, kT=0.01, FP64",
            "value": P1.n_nodes / t1, "unit": "nodes/s", "nodes": P1.n_nodes, "launch_ms": t1 * 1e3,
            "alg_bytes": b1, "achieved_GBs": b1 / t1 / 1e9, "frac_hbm_peak": b1 / t1 / 1e9 / HBM_PEAK_GBS,
            "launch": {"lanes_per_node": shape1[0], "workgroups_per_cu": shape1[1]},
            "accuracy": accuracy(base, 1, rho1.cpu().numpy())}
        p1.close()
        print(f"[bench] C1 {P1.n_nodes / t1:.1f} nodes/s", file=sys.stderr, flush=True)
    if "c3" in legs:
        # uneven batching: 20000 nodes with radii U{6..12} bohr and depths U{40..100} in one
        # persistent, autotuned, graph-replayed launch
        P3 = synth.make_problem(3)
        p3, rho3, t3, shape3, in3, _ = forward_leg(sgq, torch, P3, stream, args.tune_nodes, warm=True)
        b3 = launch_bytes(P3)
        costs = [alg_bytes(int(n), int(k)) for n, k in zip(cube_points(P3.half_width, P3.n), P3.depth)]
        configs["c3"] = {
            "workload": "96^3 grid h=0.5, 760 atoms with KB projectors, 20000 nodes, radii "
                        "U{6..12} bohr (cubes 25^3..49^3), depths U{40..100}, kT=0.005, FP32",
            "value": P3.n_nodes / t3, "unit": "nodes/s", "nodes": P3.n_nodes, "launch_ms": t3 * 1e3,
            "alg_bytes": b3, "achieved_GBs": b3 / t3 / 1e9, "frac_hbm_peak": b3 / t3 / 1e9 / HBM_PEAK_GBS,
            "node_cost_spread": max(costs) / min(costs),
            "launch": {"lanes_per_node": shape3[0], "workgroups_per_cu": shape3[1],
                       "autotuned": True, "hip_graph": True},
            "accuracy": accuracy(base, 3, rho3.cpu().numpy())}
        p3.close()
        del in3, rho3
        print(f"[bench] C3 {P3.n_nodes / t3:.1f} nodes/s", file=sys.stderr, flush=True)
    for cfg, leg, kind_name in ((4, "c4", "differentiation"), (5, "c5", "dislocation")):
        if leg not in legs:
            continue
        # every node of the workload: forward (density, for the accuracy check), the band
        # free energy, its adjoint with the Lanczos vectors recomputed, and the adjoint after
        # a forward call that checkpointed the bases of the costliest nodes within a budget
        Pk = synth.make_problem(cfg)
        if cfg == 4 and 0 < args.adjoint_nodes < Pk.n_nodes:
            Pk = Pk.subset(np.sort(np.random.default_rng(8).choice(Pk.n_nodes, args.adjoint_nodes,
                                                                   replace=False)))
        pk, rhok, tk, shapek, (vk, Rk, Ek, wk), _ = forward_leg(sgq, torch, Pk, stream, args.tune_nodes)
        acc = accuracy(base, cfg, rhok.cpu().numpy()) if Pk.n_nodes == base_nodes(cfg) else None
        del rhok
        bk = launch_bytes(Pk)
        pk.prepare_backward()
        ek = torch.empty(Pk.n_nodes, dtype=torch.float64, device="cuda")
        omk = torch.empty(1, dtype=torch.float64, device="cuda")
        g = torch.ones(1, dtype=torch.float64, device="cuda")
        dV = torch.empty_like(vk)
        dR = torch.zeros_like(Rk)
        dE = torch.zeros_like(Ek)

        def energy():
            sgq.band_energy(pk, vk, Rk, Ek, wk, Pk.mu, Pk.kT, sgq.SGQ_FREE, ek, omk,
                            stream=stream.cuda_stream)

        def backward():
            sgq.band_energy_backward(pk, vk, Rk, Ek, wk, Pk.mu, Pk.kT, sgq.SGQ_FREE, g, dV, dR, dE,
                                     stream=stream.cuda_stream)

        ta = event_time(stream, backward)
        assert pk.status() == sgq.SGQ_OK
        npts = cube_points(Pk.half_width, Pk.n)
        # algorithmic bytes of one node's adjoint: the forward recompute B(n, K), the adjoint
        # vectors and their matvec 4n*8K, the node's dV cube 4n
        abytes = float(sum(alg_bytes(int(n), int(k)) + 4.0 * int(n) * (8 * int(k) + 1)
                           for n, k in zip(npts, Pk.depth)))
        entry = {
            "forward": {"value": Pk.n_nodes / tk, "unit": "nodes/s", "launch_ms": tk * 1e3,
                        "alg_bytes": bk, "achieved_GBs": bk / tk / 1e9,
                        "frac_hbm_peak": bk / tk / 1e9 / HBM_PEAK_GBS,
                        "launch": {"lanes_per_node": shapek[0], "workgroups_per_cu": shapek[1]},
                        "accuracy": acc},
            "adjoint": {"value": Pk.n_nodes / ta, "unit": "nodes/s", "s": ta, "alg_bytes": abytes,
                        "achieved_GBs": abytes / ta / 1e9,
                        "frac_hbm_peak": abytes / ta / 1e9 / HBM_PEAK_GBS,
                        "recompute": True}}
        if args.retain_gb > 0:
            dV_re = dV.clone()
            free_b, _ = torch.cuda.mem_get_info()
            budget = int(min(args.retain_gb * 1e9, free_b - 24e9))
            try:
                n_ret = pk.set_retain(True, max_bytes=budget) if budget > 0 else 0
            except sgq.SgqError as err:
                n_ret = 0
                print(f"[bench] no checkpointed adjoint: {err}", file=sys.stderr, flush=True)
            if n_ret > 0:
                tf = event_time(stream, energy)
                tb = event_time(stream, backward)
                assert pk.status() == sgq.SGQ_OK
                entry["adjoint"]["checkpointed"] = {
                    "value": Pk.n_nodes / tb, "unit": "nodes/s", "s": tb,
                    "retained_nodes": n_ret, "budget_GB": budget / 1e9, "forward_s": tf,
                    "forward_plus_backward_nodes_per_s": Pk.n_nodes / (tf + tb),
                    "forward_plus_recompute_backward_nodes_per_s": Pk.n_nodes / (tk + ta),
                    # the forward ran with the autotuned lanes per node and the recompute
                    # with the backward's, which follow each node's cube: where the two
                    # differ, so do the gradients, by FP32 rounding only
                    "dV_normwise_rel_diff_vs_recompute":
                        float((dV - dV_re).abs().max() / dV_re.abs().max())}
                print(f"[bench] C{cfg} checkpointed adjoint {Pk.n_nodes / tb:.1f} nodes/s "
                      f"({n_ret} of {Pk.n_nodes} nodes retained)", file=sys.stderr, flush=True)
            pk.set_retain(False)
            del dV_re
        if cfg == 4:
            which = ("all 110592 grid points" if Pk.n_nodes == 110592 else
                     f"{Pk.n_nodes} seeded grid points")
            entry["workload"] = (f"48^3 grid h=0.5, 16 atoms with KB projectors, {which} as "
                                 "nodes, 33^3 cubes, K=60, kT=0.01, FP32; adjoint "
                                 "dOmega/dV + dOmega/dR + dOmega/dE of the Mermin free energy")
        else:
            entry["workload"] = ("128^3 grid h=0.5, 1925 screw-displaced atoms with KB projectors, "
                                 "all 65536 nodes (weights 32), cubes 25^3..49^3, K=80, kT=0.005, "
                                 "FP32; adjoint of the Mermin free energy")
        configs[leg] = entry
        pk.close()
        del vk, Rk, Ek, wk, dV, dR, dE, ek
        torch.cuda.empty_cache()
        print(f"[bench] C{cfg} fwd {Pk.n_nodes / tk:.1f} adj {Pk.n_nodes / ta:.1f} nodes/s",
              file=sys.stderr, flush=True)
    if configs:
        rec["configs"] = configs
    if base is not None:
        rec["cpu_baseline"] = cpu_record(base, 2, "the 8192-node 64^3 workload")
        rec["cpu_baseline"]["next_rows"] = oracle_rows
        rec["cpu_baseline"]["configs"] = {
            f"c{c}": cpu_record(base, c, d) for c, d in
            ((1, "the 16^3 untruncated FP64 workload"), (3, "the 20000-node 96^3 workload"),
             (4, "the 110592-node 48^3 workload"), (5, "the 65536-node 128^3 workload"))
            if c in base}
        rec["accuracy"] = accuracy(base, 2, rho_c2)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
