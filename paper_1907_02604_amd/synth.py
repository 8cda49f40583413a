"""Seeded synthetic inputs for the spectral-quadrature density path.

This module only *draws* inputs: atom sites, the local potential grid, projector
energies and the node list (centres, truncation half-widths, Lanczos depths, weights).
It contains none of the quadrature arithmetic, so both the HIP library's tests and
the FP64 oracle may consume what it produces.

Inputs stand in for the Mg systems of the paper's Sec. "Computational set-up"
(hcp Mg, screw dislocations); the paper's own pseudopotential and meshes are not
available, so a Gaussian local potential on a jittered hcp lattice is used instead.

Conventions
-----------
* Global grid: ``n = (nx, ny, nz)`` points, spacing ``h`` (bohr), periodic box
  ``L = n*h``.  Arrays are stored C-ordered as ``[z, y, x]`` so that x is the
  fastest index; the linear index of grid point (ix, iy, iz) is
  ``ix + nx*(iy + ny*iz)``.
* Atom positions ``R`` are Cartesian (x, y, z) in bohr, wrapped into ``[0, L)``.
* Node half-width ``R_q`` is in grid points (cube side ``2*R_q + 1``); ``-1`` means
  the untruncated periodic Hamiltonian on the whole grid.

Random draw order (``numpy.random.default_rng(seed)``): jitter (M x 3 normal),
projector energies (M x 4 uniform), node centres (choice without replacement),
radii, depths; a config skips the draws it does not need (all-node configs draw no
centres, fixed-radius configs no radii, fixed-depth configs no depths).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

HCP_A = 6.06            # bohr
HCP_C_OVER_A = 1.624
VLOC_DEPTH = -2.0       # Ha
VLOC_SIGMA = 1.0        # bohr
VLOC_CUTOFF_SIGMAS = 8.0
PROJ_RC = 1.5           # bohr
PROJ_RG = 0.5           # bohr
N_PROJ = 4              # s, px, py, pz


@dataclasses.dataclass
class Problem:
    name: str
    n: tuple            # (nx, ny, nz)
    h: float
    atoms: np.ndarray   # (M, 3) float64, bohr
    proj_E: np.ndarray  # (M, 4) float64, Ha (all zero when n_proj == 0)
    n_proj: int         # 0 or 4
    v_loc: np.ndarray   # (nz, ny, nx) float64, Ha
    centers: np.ndarray     # (Nq,) int64 linear grid index
    half_width: np.ndarray  # (Nq,) int32, grid points, -1 = untruncated periodic
    depth: np.ndarray       # (Nq,) int32, Lanczos depth K
    weight: np.ndarray      # (Nq,) float64, node weight n_q
    mu: float
    kT: float
    precision: str          # "f64" or "f32"
    seed: int

    @property
    def L(self):
        return tuple(ni * self.h for ni in self.n)

    @property
    def n_nodes(self):
        return int(self.centers.shape[0])

    def subset(self, idx):
        """Same system restricted to the nodes ``idx`` (order kept)."""
        idx = np.asarray(idx, dtype=np.int64)
        return dataclasses.replace(
            self, centers=self.centers[idx].copy(), half_width=self.half_width[idx].copy(),
            depth=self.depth[idx].copy(), weight=self.weight[idx].copy())


def hcp_sites(L, a=HCP_A, c_over_a=HCP_C_OVER_A):
    """Sites of an orthohexagonal hcp lattice (cell a x sqrt(3)a x c, 4-site basis)
    lying in the half-open box [0, L)^3.  Order: cell index (i, j, k) then basis."""
    c = a * c_over_a
    cell = np.array([a, math.sqrt(3.0) * a, c])
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 1.0 / 6.0, 0.5], [0.0, 2.0 / 3.0, 0.5]])
    L = np.asarray(L, dtype=np.float64)
    counts = np.ceil(L / cell).astype(int) + 1
    out = []
    for i in range(-1, counts[0]):
        for j in range(-1, counts[1]):
            for k in range(-1, counts[2]):
                for b in basis:
                    p = (np.array([i, j, k], dtype=np.float64) + b) * cell
                    if np.all(p >= 0.0) and np.all(p < L):
                        out.append(p)
    return np.array(out, dtype=np.float64).reshape(-1, 3)


def screw_displace(sites, L, b=HCP_A):
    """Volterra screw along z through the box centre: u_z = b*theta/(2*pi),
    theta = atan2(y - Ly/2, x - Lx/2) in (-pi, pi]."""
    out = sites.copy()
    theta = np.arctan2(sites[:, 1] - L[1] / 2.0, sites[:, 0] - L[0] / 2.0)
    out[:, 2] = sites[:, 2] + b * theta / (2.0 * math.pi)
    return out


def gaussian_vloc(n, h, atoms, depth=VLOC_DEPTH, sigma=VLOC_SIGMA, cutoff=VLOC_CUTOFF_SIGMAS):
    """V(x) = depth * sum_J sum_images exp(-|x - R_J - L m|^2 / (2 sigma^2)),
    keeping every image term with |x - R_J - L m| <= cutoff*sigma.  FP64, [z, y, x]."""
    n = tuple(int(v) for v in n)
    nx, ny, nz = n
    rcut = cutoff * sigma
    w = int(math.ceil(rcut / h)) + 1
    offs = np.arange(-w, w + 1)
    total = np.zeros(nx * ny * nz, dtype=np.float64)
    chunk = 32
    for J0 in range(0, atoms.shape[0], chunk):
        R = atoms[J0:J0 + chunk]
        g = np.floor(R / h).astype(np.int64)                  # (m, 3)
        ix = g[:, 0:1] + offs                                  # (m, W)
        iy = g[:, 1:2] + offs
        iz = g[:, 2:3] + offs
        dx = ix * h - R[:, 0:1]
        dy = iy * h - R[:, 1:2]
        dz = iz * h - R[:, 2:3]
        r2 = (dz[:, :, None, None] ** 2 + dy[:, None, :, None] ** 2
              + dx[:, None, None, :] ** 2)
        val = np.where(r2 <= rcut * rcut, np.exp(-r2 / (2.0 * sigma * sigma)), 0.0)
        lin = (np.mod(ix, nx)[:, None, None, :]
               + nx * (np.mod(iy, ny)[:, None, :, None] + ny * np.mod(iz, nz)[:, :, None, None]))
        total += np.bincount(lin.ravel(), weights=val.ravel(), minlength=total.size)
    return (depth * total).reshape(nz, ny, nx)


def _base(name, N, h, seed, *, screw=False, keep_nearest=None):
    L = (N * h,) * 3
    sites = hcp_sites(L)
    if keep_nearest is not None:
        centre = np.array(L) / 2.0
        dist = np.linalg.norm(sites - centre, axis=1)
        order = np.argsort(dist, kind="stable")
        sites = sites[np.sort(order[:keep_nearest])]
    if screw:
        sites = screw_displace(sites, L)
    rng = np.random.default_rng(seed)
    jitter = rng.normal(0.0, 0.05, size=sites.shape)
    atoms = np.mod(sites + jitter, np.array(L))
    proj_E = rng.uniform(-1.0, 1.0, size=(atoms.shape[0], N_PROJ))
    return rng, atoms, proj_E


def make_problem(cfg, *, n_nodes=None, grid=None):
    """Build config ``cfg`` in 1..5 (the five workloads of the benchmark set).

    ``n_nodes`` overrides the node count of sampled configs (a smaller seeded
    sample of the same distribution); ``grid`` overrides N for tests."""
    h = 0.5
    if cfg == 1:
        N = grid or 16
        rng, atoms, E = _base("C1", N, h, 1)
        nn = N ** 3
        centers = np.arange(nn, dtype=np.int64)
        hw = np.full(nn, -1, np.int32)
        K = np.full(nn, 30, np.int32)
        return Problem("C1 16^3 periodic FP64 K=30", (N,) * 3, h, atoms, np.zeros_like(E), 0,
                       gaussian_vloc((N,) * 3, h, atoms), centers, hw, K, np.ones(nn), -0.1, 0.01,
                       "f64", 1)
    if cfg == 2:
        N = grid or 64
        rng, atoms, E = _base("C2", N, h, 2)
        nq = n_nodes or 8192
        centers = rng.choice(N ** 3, size=nq, replace=False).astype(np.int64)
        hw = np.full(nq, 16, np.int32)
        K = np.full(nq, 60, np.int32)
        return Problem("C2 64^3 33^3-cube K=60 KB FP32", (N,) * 3, h, atoms, E, 4,
                       gaussian_vloc((N,) * 3, h, atoms), centers, hw, K, np.ones(nq), -0.1, 0.01,
                       "f32", 2)
    if cfg == 3:
        N = grid or 96
        rng, atoms, E = _base("C3", N, h, 3)
        nq = n_nodes or 20000
        centers = rng.choice(N ** 3, size=nq, replace=False).astype(np.int64)
        radii = rng.integers(6, 13, size=nq)
        depths = rng.integers(40, 101, size=nq)
        hw = (radii * 2).astype(np.int32)     # r / h with h = 0.5
        return Problem("C3 96^3 uneven cubes 25^3..49^3 K=40..100 KB FP32", (N,) * 3, h, atoms, E,
                       4, gaussian_vloc((N,) * 3, h, atoms), centers, hw, depths.astype(np.int32),
                       np.ones(nq), -0.1, 0.005, "f32", 3)
    if cfg == 4:
        N = grid or 48
        rng, atoms, E = _base("C4", N, h, 4, keep_nearest=16)
        nn = N ** 3
        centers = np.arange(nn, dtype=np.int64)
        hw = np.full(nn, 16, np.int32)
        K = np.full(nn, 60, np.int32)
        return Problem("C4 48^3 16 atoms all nodes 33^3 K=60 KB FP32", (N,) * 3, h, atoms, E, 4,
                       gaussian_vloc((N,) * 3, h, atoms), centers, hw, K, np.ones(nn), -0.1, 0.01,
                       "f32", 4)
    if cfg == 5:
        N = grid or 128
        rng, atoms, E = _base("C5", N, h, 5, screw=True)
        nq = n_nodes or 65536
        centers = rng.choice(N ** 3, size=nq, replace=False).astype(np.int64)
        radii = rng.integers(6, 13, size=nq)
        hw = (radii * 2).astype(np.int32)
        K = np.full(nq, 80, np.int32)
        w = np.full(nq, (N ** 3) / 65536.0)
        return Problem("C5 128^3 screw 65536 nodes 25^3..49^3 K=80 KB FP32", (N,) * 3, h, atoms,
                       E, 4, gaussian_vloc((N,) * 3, h, atoms), centers, hw, K, w, -0.1, 0.005,
                       "f32", 5)
    raise ValueError(f"unknown config {cfg}")


def grid_coords(linear, n):
    """(ix, iy, iz) of linear grid indices."""
    nx, ny, _ = n
    linear = np.asarray(linear, dtype=np.int64)
    return linear % nx, (linear // nx) % ny, linear // (nx * ny)


# ------------------------------------------------------------------ coarse-grained inputs
def coarse_esps(n, seed, n_sampled, zone_radius):
    """Energy/electronic sampling points of a coarse-grained run: every grid point within
    `zone_radius` grid points of the box-centre line along z (the full-resolution zone
    around a dislocation core) plus `n_sampled` seeded uniform grid points.  Ascending
    unique linear indices."""
    nx, ny, nz = n
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    disk = ((ix - nx // 2) ** 2 + (iy - ny // 2) ** 2 <= zone_radius ** 2).ravel()
    plane = np.nonzero(disk)[0].astype(np.int64)           # ix + nx*iy
    zone = (plane[None, :] + nx * ny * np.arange(nz, dtype=np.int64)[:, None]).ravel()
    rng = np.random.default_rng(seed)
    sampled = rng.choice(nx * ny * nz, size=n_sampled, replace=False).astype(np.int64)
    return np.unique(np.concatenate([zone, sampled]))


def esp_mesh(n, esp_center):
    """Tetrahedral mesh over the ESPs: the Delaunay tetrahedralisation (qhull through
    scipy) of their unwrapped grid coordinates, with the zero-volume tetrahedra that
    degenerate (coplanar / cospherical) lattice points produce removed.  The kept
    tetrahedra tile the convex hull; their orientations are mixed, as qhull returns them.
    int32 (T, 4) ESP indices."""
    from scipy.spatial import Delaunay
    nx, ny, _ = n
    c = np.asarray(esp_center, dtype=np.int64)
    xyz = np.stack([c % nx, (c // nx) % ny, c // (nx * ny)], axis=1)
    tets = Delaunay(xyz.astype(np.float64)).simplices.astype(np.int64)
    v = xyz[tets]
    a, b, d = v[:, 1] - v[:, 0], v[:, 2] - v[:, 0], v[:, 3] - v[:, 0]
    vol6 = np.einsum("ij,ij->i", a, np.cross(b, d))
    return tets[vol6 != 0].astype(np.int32)


def predictor_fields(n, h, sites, sigma=1.2):
    """Two smooth synthetic predictor fields on the grid, (2, nz, ny, nx) FP64: a
    density-like sum of Gaussians 0.05 exp(-r^2/2 sigma^2) at `sites` (the undisplaced
    lattice of the defect-free crystal) and a potential-like sum -0.8 exp(-r^2/2 s^2)
    with s = 1.5 sigma; each Gaussian is cut at 4 of its widths."""
    rho0 = gaussian_vloc(n, h, sites, depth=0.05, sigma=sigma, cutoff=4.0)
    phi0 = gaussian_vloc(n, h, sites, depth=-0.8, sigma=1.5 * sigma, cutoff=4.0)
    return np.stack([rho0, phi0])


def nuclear_charge(n, h, atoms, Z=2.0, sigma=0.8):
    """Regularised nuclear charge density b(x) = -Z sum_J g(x - R_J) on the grid, (nz, ny, nx)
    FP64, with g the unit-mass Gaussian of width sigma (bohr), periodic images within 6
    widths.  Z = 2 stands for the two valence electrons of magnesium."""
    norm = -Z / ((2.0 * math.pi) ** 1.5 * sigma ** 3)
    return gaussian_vloc(n, h, atoms, depth=norm, sigma=sigma, cutoff=6.0)
