"""Small problem builders shared by the oracle pin tests (CPU only)."""
import numpy as np

from paper_1907_02604_amd import synth


def custom_problem(N, h=0.5, atoms=None, proj_E=None, v_loc=None, centers=None, half_width=-1,
                   depth=10, weight=1.0, mu=-0.1, kT=0.01, n_proj=None):
    atoms = np.zeros((0, 3)) if atoms is None else np.asarray(atoms, dtype=np.float64)
    if proj_E is None:
        proj_E = np.zeros((atoms.shape[0], 4))
    if n_proj is None:
        n_proj = 4 if np.any(proj_E != 0) else 0
    if v_loc is None:
        v_loc = np.zeros((N, N, N))
    if centers is None:
        centers = np.arange(N ** 3)
    centers = np.asarray(centers, dtype=np.int64)
    nq = centers.size
    return synth.Problem("custom", (N, N, N), h, atoms, np.asarray(proj_E, dtype=np.float64),
                         n_proj, v_loc, centers, np.full(nq, half_width, np.int32),
                         np.full(nq, depth, np.int32), np.full(nq, float(weight)), mu, kT, "f64", 0)


def smooth_random_potential(N, seed, amp=1.0):
    """A smooth random periodic field (few low Fourier modes), (z, y, x)."""
    rng = np.random.default_rng(seed)
    x = np.arange(N) * 2 * np.pi / N
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    v = np.zeros((N, N, N))
    for _ in range(4):
        k = rng.integers(0, 3, size=3)
        ph = rng.uniform(0, 2 * np.pi)
        v += rng.normal() * np.cos(k[0] * X + k[1] * Y + k[2] * Z + ph)
    return amp * v


def lin(ix, iy, iz, N):
    return ix + N * (iy + N * iz)


_POOL_PROBLEM = None


def _pool_init(prob):
    global _POOL_PROBLEM
    from threadpoolctl import threadpool_limits
    threadpool_limits(1)              # one BLAS thread per worker process
    _POOL_PROBLEM = prob


def _pool_node(q):
    import oracle as O
    return float(O.rho_quadrature(_POOL_PROBLEM, nodes=[int(q)])[0][0])


def oracle_rho_pool(prob, nodes, workers=16):
    """Oracle densities of the listed nodes on a pool of spawned worker processes (they
    import only the oracle and the input generator, never the GPU runtime), at most
    `workers` of them and no more than the host's cores."""
    import multiprocessing as mp
    import os
    n = max(1, min(workers, len(os.sched_getaffinity(0)), len(nodes)))
    with mp.get_context("spawn").Pool(n, initializer=_pool_init, initargs=(prob,)) as pool:
        return np.array(pool.map(_pool_node, [int(q) for q in nodes], chunksize=1))


def per_node_rel_err(got, ref, floor=1e-3):
    """Largest per-node relative error over the nodes whose reference exceeds floor times
    the largest |reference| (the per-node companion of the normwise metric)."""
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    sig = np.abs(ref) > floor * np.max(np.abs(ref))
    return float(np.max(np.abs(got[sig] - ref[sig]) / np.abs(ref[sig])))
