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
