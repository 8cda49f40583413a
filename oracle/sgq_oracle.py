"""Plain FP64 CPU oracle for the spectral Gauss-quadrature electron density.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or run
this module; only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` use it.  It shares no code with the HIP library: the only
common module is the seeded input generator ``paper_1907_02604_amd.synth``, which
holds no quadrature arithmetic.

What it computes (paper: Sec. "Density Functional Theory"):

* the Fermi-Dirac density matrix gamma = g(H; mu), g = 1/(1+exp((lam-mu)/kT))
  (Eq. eq:dm);
* for every node p the K-point Gauss rule (lambda_k, w_k) of the spectral measure
  of H contracted with the FD basis function eta_p (Eq. eq:9), obtained by a
  K-step Lanczos iteration started from eta_p (paragraph after Eq.
  Eqn:LSSGQ:Electron_density:GQ) and the eigen-decomposition of the Lanczos
  tridiagonal (nodes = eigenvalues, weights = squared first eigenvector
  components);
* rho_p = 2 h^-3 sum_k w_k g(lambda_k) (Eq. Eqn:LSSGQ:Electron_density:GQ);
* the per-node band / free-energy term e_p = 2 sum_k w_k F(lambda_k) (the first and
  last terms of Eq. eq:tot) and the weighted sum Omega = sum_q n_q e_q
  (Eq. eq:free_cg);
* the exact-arithmetic adjoint of Omega with respect to the local potential,
  the projector energies and the atom positions (reverse mode through the
  Lanczos three-term recurrence and the Daleckii-Krein derivative of F(T));
* the Fermi level: the mu at which the electron count of the stored rules,
  N(mu) = 2 sum_q n_q sum_k w_k g(theta_k; mu) (Eq. Eqn:LSSGQ:Fermi_level:GQ with
  the node weights of Eq. eq:free_cg), equals a given N_e;
* the cluster-sampled energy E = sum_q n_q Fbar_q, Fbar_q the mean per-point energy
  over the grid points within a radius of ESP q (Eq. eq:free_cg_sampling);
* the predictor + corrector reconstruction of fields on the fine grid: the corrector
  at the ESPs interpolated by the linear shape functions of a tetrahedral mesh over
  the ESPs and added to the predictor (Eq. eq:pc, Eq. phi_approx_scheme).
* the self-consistency ingredients: the LDA exchange-correlation energy and potential
  (Eq. eq:xc, Perdew-Wang correlation) and the periodic Poisson solve for the
  electrostatic potential with the FD Laplacian (Eq. eq:poisson), and their sum, the
  potential of the Hamiltonian (Eq. Eqn:Hamiltonian).

Everything is float64 and written for readability, not speed: one node at a
time, numpy array ops for the stencil, a library tridiagonal eigensolver.

Readings where the paper is silent:
* H = -1/2 Lap_6 + V_loc + V_nl on the grid, where Lap_6 is the sixth-order
  central finite-difference Laplacian applied axis by axis (no cross terms);
* node truncation: H_q = P_q H P_q on a cube of side 2R+1 centred at the node,
  indices wrapping periodically into the global grid, zero outside the cube;
  R = -1 means the untruncated periodic Hamiltonian;
* start vector = unit vector at the node (the orthonormal FD basis function);
* full classical Gram-Schmidt reorthogonalisation each step, repeated once when
  the norm drops by more than 1/sqrt(2); breakdown when beta <= tau * scale with
  scale = 9.0667/h^2 + max|V|, after which the rule has K_eff < K nodes and is exact;
* integrands F: BAND F = lam*g; FREE (Mermin) F = lam*g + kT[g ln g + (1-g) ln(1-g)]
  = mu*g - kT*softplus(-(lam-mu)/kT); GRAND F = -kT*softplus(-(lam-mu)/kT);
* cluster sampling: N in the cluster average is the number of grid points of the ball,
  the ball is closed with minimum-image distances, and membership is decided on the
  integer squared distance against (r/h)^2 (1 + 1e-9);
* corrector interpolation: linear shape functions on a tetrahedral mesh over the ESPs
  (grid points, unwrapped coordinates); a point takes the lowest-numbered tetrahedron
  holding it, zero-volume tetrahedra are skipped, points in none keep the predictor;
* exchange-correlation: the Perdew-Wang (1992) unpolarised parametrisation of the
  correlation energy, zero energy and potential where rho <= 0;
* Poisson: the periodic problem with the Hamiltonian's FD Laplacian, the mean of the
  source removed (and reported), phi of zero mean.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.integrate
import scipy.linalg
import scipy.optimize
import scipy.sparse

BAND, FREE, GRAND = 0, 1, 2

# Sixth-order central weights of d^2/dx^2 for offsets 0, +-1, +-2, +-3 (times 1/h^2).
FD2_WEIGHTS = (-49.0 / 18.0, 3.0 / 2.0, -3.0 / 20.0, 1.0 / 90.0)

TAU_FP64 = 1e-12


# --------------------------------------------------------------------------------------
# Fermi-Dirac occupation and integrands (Eq. eq:dm, Eq. eq:tot)
# --------------------------------------------------------------------------------------
def fermi(lam, mu, kT):
    """g(lam) = 1/(1 + exp((lam - mu)/kT)), evaluated without overflow."""
    x = (np.asarray(lam, dtype=np.float64) - mu) / kT
    out = np.empty_like(x)
    pos = x > 0
    e = np.exp(-x[pos])
    out[pos] = e / (1.0 + e)
    out[~pos] = 1.0 / (1.0 + np.exp(x[~pos]))
    return out


def softplus(x):
    """ln(1 + exp(x)) without overflow."""
    x = np.asarray(x, dtype=np.float64)
    return np.maximum(x, 0.0) + np.log1p(np.exp(-np.abs(x)))


def integrand(lam, mu, kT, kind):
    """F(lam) for the per-node energy e = 2 sum_k w_k F(lam_k)."""
    lam = np.asarray(lam, dtype=np.float64)
    g = fermi(lam, mu, kT)
    if kind == BAND:
        return lam * g
    sp = kT * softplus(-(lam - mu) / kT)
    if kind == FREE:
        return mu * g - sp
    if kind == GRAND:
        return -sp
    raise ValueError(kind)


def integrand_deriv(lam, mu, kT, kind):
    """dF/dlam."""
    lam = np.asarray(lam, dtype=np.float64)
    g = fermi(lam, mu, kT)
    dg = -g * (1.0 - g) / kT
    if kind == BAND:
        return g + lam * dg
    if kind == FREE:
        return g + mu * dg
    if kind == GRAND:
        return g
    raise ValueError(kind)


def divided_differences(theta, mu, kT, kind):
    """D[k, l] = (F(theta_k) - F(theta_l)) / (theta_k - theta_l), F'(midpoint) when the
    two nodes are closer than 1e-6*max(kT, |theta|)."""
    theta = np.asarray(theta, dtype=np.float64)
    F = integrand(theta, mu, kT, kind)
    a = theta[:, None]
    b = theta[None, :]
    diff = a - b
    close = np.abs(diff) <= 1e-6 * np.maximum(kT, np.maximum(np.abs(a), np.abs(b)))
    safe = np.where(close, 1.0, diff)
    D = (F[:, None] - F[None, :]) / safe
    mid = integrand_deriv(0.5 * (a + b), mu, kT, kind)
    return np.where(close, mid, D)


# --------------------------------------------------------------------------------------
# Kleinman-Bylander projectors (s, px, py, pz Gaussians with a smooth cutoff)
# --------------------------------------------------------------------------------------
def projector_norms(rg, rc):
    """Continuum normalisation constants (N_s, N_p) so that the integral of chi^2
    over R^3 is one for every channel."""
    def cut(r):
        return (1.0 - (r / rc) ** 2) ** 3

    def gs(r):
        return math.exp(-r * r / (2.0 * rg * rg)) * cut(r)

    i_s = scipy.integrate.quad(lambda r: 4.0 * math.pi * r * r * gs(r) ** 2, 0.0, rc,
                               epsabs=0, epsrel=1e-13, limit=200)[0]
    # p_x = (x/rg) g c; angular average of x^2 is r^2/3
    i_p = scipy.integrate.quad(lambda r: 4.0 * math.pi * r * r * (r * r / (3.0 * rg * rg)) * gs(r) ** 2,
                               0.0, rc, epsabs=0, epsrel=1e-13, limit=200)[0]
    return 1.0 / math.sqrt(i_s), 1.0 / math.sqrt(i_p)


def projector_values(d, rg, rc, norms):
    """chi_l(d) for displacement d = x - R_J (..., 3) bohr -> (..., 4): s, px, py, pz."""
    Ns, Np = norms
    d = np.asarray(d, dtype=np.float64)
    r2 = np.sum(d * d, axis=-1)
    inside = r2 < rc * rc
    g = np.exp(-r2 / (2.0 * rg * rg)) * np.where(inside, (1.0 - r2 / (rc * rc)) ** 3, 0.0)
    out = np.empty(d.shape[:-1] + (4,))
    out[..., 0] = Ns * g
    for a in range(3):
        out[..., 1 + a] = Np * (d[..., a] / rg) * g
    return out


def projector_gradients(d, rg, rc, norms):
    """d chi_l / d d_a for displacement d (..., 3) -> (..., 4, 3).  (d chi/d R = -this.)"""
    Ns, Np = norms
    d = np.asarray(d, dtype=np.float64)
    r2 = np.sum(d * d, axis=-1)
    inside = r2 < rc * rc
    e = np.exp(-r2 / (2.0 * rg * rg))
    t = np.where(inside, 1.0 - r2 / (rc * rc), 0.0)
    g = e * t ** 3
    # d g / d d_a = d_a * e * [ -t^3 / rg^2 - 6 t^2 / rc^2 ]
    dg_over_d = e * (-(t ** 3) / (rg * rg) - 6.0 * t * t / (rc * rc))
    out = np.empty(d.shape[:-1] + (4, 3))
    for a in range(3):
        out[..., 0, a] = Ns * dg_over_d * d[..., a]
    for l in range(3):
        for a in range(3):
            val = Np / rg * d[..., l] * dg_over_d * d[..., a]
            if l == a:
                val = val + Np / rg * g
            out[..., 1 + l, a] = val
    return out


# --------------------------------------------------------------------------------------
# The node Hamiltonian H_q (Eq. Eqn:Hamiltonian discretised on the FD grid)
# --------------------------------------------------------------------------------------
def kinetic_apply(v, h, periodic):
    """-1/2 Lap_6 v on a (z, y, x) array; zero outside the box unless periodic."""
    out = 3.0 * FD2_WEIGHTS[0] * v
    for axis in range(3):
        for d in (1, 2, 3):
            wgt = FD2_WEIGHTS[d]
            if periodic:
                out = out + wgt * (np.roll(v, d, axis=axis) + np.roll(v, -d, axis=axis))
            else:
                fwd = np.zeros_like(v)
                bwd = np.zeros_like(v)
                src = [slice(None)] * 3
                dst = [slice(None)] * 3
                src[axis] = slice(0, v.shape[axis] - d)
                dst[axis] = slice(d, v.shape[axis])
                fwd[tuple(dst)] = v[tuple(src)]      # fwd[i] = v[i - d]
                bwd[tuple(src)] = v[tuple(dst)]      # bwd[i] = v[i + d]
                out = out + wgt * (fwd + bwd)
    return (-0.5 / (h * h)) * out


def kinetic_gershgorin(h):
    """Gershgorin bound of -1/2 Lap_6: 3 * 1/2 * (49/18 + 2*(3/2 + 3/20 + 1/90)) / h^2."""
    return 1.5 * (abs(FD2_WEIGHTS[0]) + 2.0 * sum(abs(w) for w in FD2_WEIGHTS[1:])) / (h * h)


class NodeHamiltonian:
    """H_q for one node of a problem (a ``synth.Problem``).

    Periodic mode (half_width < 0): the whole grid, periodic stencil, the start
    vector at the node.  Truncated mode: the cube of side s = 2R+1 around the node,
    grid indices wrapping periodically, Dirichlet zero outside; requires
    s <= n_a - 6 on every axis so that no coupling of H wraps around the cube."""

    def __init__(self, prob, node, v_loc=None, atoms=None, proj_E=None):
        self.h = float(prob.h)
        nx, ny, nz = prob.n
        v_loc = prob.v_loc if v_loc is None else v_loc
        self.atoms = prob.atoms if atoms is None else atoms
        self.proj_E = prob.proj_E if proj_E is None else proj_E
        self.n_proj = int(prob.n_proj)
        c = int(prob.centers[node])
        cx, cy, cz = c % nx, (c // nx) % ny, c // (nx * ny)
        R = int(prob.half_width[node])
        self.periodic = R < 0
        if self.periodic:
            self.shape = (nz, ny, nx)
            self.origin = (0, 0, 0)
            self.start = (cz, cy, cx)
            self.gz = np.arange(nz)
            self.gy = np.arange(ny)
            self.gx = np.arange(nx)
        else:
            s = 2 * R + 1
            if s > min(nx, ny, nz) - 6:
                raise ValueError("cube side exceeds grid size - 6")
            self.shape = (s, s, s)
            self.origin = (cz - R, cy - R, cx - R)
            self.start = (R, R, R)
            self.gz = np.mod(cz - R + np.arange(s), nz)
            self.gy = np.mod(cy - R + np.arange(s), ny)
            self.gx = np.mod(cx - R + np.arange(s), nx)
        self.grid_n = (nz, ny, nx)
        self.v = v_loc[np.ix_(self.gz, self.gy, self.gx)]
        self.scale = kinetic_gershgorin(self.h) + float(np.max(np.abs(v_loc)))
        self._build_projectors()

    # -- projector columns restricted to the cube -----------------------------------
    def _local_index(self, gz, gy, gx):
        """Flat local index of global points, or -1 when outside the cube."""
        nz, ny, nx = self.grid_n
        if self.periodic:
            return (np.mod(gz, nz) * ny + np.mod(gy, ny)) * nx + np.mod(gx, nx)
        s = self.shape[0]
        lz = np.mod(gz - self.origin[0], nz)
        ly = np.mod(gy - self.origin[1], ny)
        lx = np.mod(gx - self.origin[2], nx)
        ok = (lz < s) & (ly < s) & (lx < s)
        return np.where(ok, (lz * s + ly) * s + lx, -1)

    def _build_projectors(self):
        self.proj_atoms = []
        self.chi = None
        if self.n_proj == 0 or self.atoms.shape[0] == 0:
            return
        h = self.h
        self.norms = projector_norms(0.5, 1.5)
        # grid points within rc of R lie within ceil(rc/h + 1/2) of the nearest grid point
        m = int(math.ceil(1.5 / h + 0.5))
        offs = np.arange(-m, m + 1)
        oz, oy, ox = np.meshgrid(offs, offs, offs, indexing="ij")
        rows, cols, vals, dvals = [], [], [], []
        col = 0
        npts = int(np.prod(self.shape))
        for J in range(self.atoms.shape[0]):
            RJ = self.atoms[J]
            g0 = np.rint(RJ / h).astype(np.int64)
            px = (g0[0] + ox).ravel()
            py = (g0[1] + oy).ravel()
            pz = (g0[2] + oz).ravel()
            disp = np.stack([px * h - RJ[0], py * h - RJ[1], pz * h - RJ[2]], axis=-1)
            chi = projector_values(disp, 0.5, 1.5, self.norms)          # (box, 4)
            dchi = projector_gradients(disp, 0.5, 1.5, self.norms)      # (box, 4, 3)
            li = self._local_index(pz, py, px)
            keep = (li >= 0) & np.any(chi != 0.0, axis=1)
            if not np.any(keep):
                continue
            self.proj_atoms.append(J)
            for l in range(4):
                rows.append(li[keep])
                cols.append(np.full(int(keep.sum()), col + l))
                vals.append(chi[keep, l])
                dvals.append(dchi[keep, l, :])
            col += 4
        if not self.proj_atoms:
            return          # no projector reaches the cube: the nonlocal sum is empty
        r = np.concatenate(rows)
        cidx = np.concatenate(cols)
        # duplicates (several images of one atom on a tiny periodic grid) are summed
        self.chi = scipy.sparse.csr_matrix((np.concatenate(vals), (r, cidx)), shape=(npts, col))
        dv = np.concatenate(dvals)
        self.dchi = [scipy.sparse.csr_matrix((dv[:, a], (r, cidx)), shape=(npts, col))
                     for a in range(3)]
        self.E_cols = np.concatenate([self.proj_E[J] for J in self.proj_atoms])

    # -- matvec -------------------------------------------------------------------
    def apply(self, vec):
        """H_q vec for a flat vector over the cube points."""
        v3 = vec.reshape(self.shape)
        out = kinetic_apply(v3, self.h, self.periodic) + self.v * v3
        out = out.ravel()
        if self.chi is not None:
            h3 = self.h ** 3
            coef = h3 * (self.chi.T @ vec)
            out = out + self.chi @ (self.E_cols * coef)
        return out

    def start_vector(self):
        e = np.zeros(self.shape)
        e[self.start] = 1.0
        return e.ravel()

    def dense(self):
        n = int(np.prod(self.shape))
        I = np.eye(n)
        return np.stack([self.apply(I[:, i]) for i in range(n)], axis=1)


# --------------------------------------------------------------------------------------
# Lanczos iteration and the Gauss rule (paragraph after Eq. Eqn:LSSGQ:Electron_density:GQ)
# --------------------------------------------------------------------------------------
def lanczos(apply_H, start, K, scale, tau=TAU_FP64):
    """K-step Lanczos from a unit start vector with full CGS reorthogonalisation.

    Returns (alpha[K_eff], beta[K_eff - 1], Q[K_eff, n], beta_last) where T_K has
    diagonal alpha and off-diagonal beta, and q_1..q_K_eff are the Lanczos vectors."""
    n = start.size
    Q = np.zeros((K, n))
    alpha = np.zeros(K)
    beta = np.zeros(K)
    q = start.astype(np.float64).copy()
    q_prev = np.zeros(n)
    b_prev = 0.0
    k_eff = K
    for j in range(K):
        Q[j] = q
        u = apply_H(q)
        a = float(q @ u)
        w = u - a * q - b_prev * q_prev
        for _ in range(2):
            before = np.linalg.norm(w)
            coef = Q[:j + 1] @ w
            w = w - Q[:j + 1].T @ coef
            if np.linalg.norm(w) >= before / math.sqrt(2.0):
                break
        b = float(np.linalg.norm(w))
        alpha[j] = a
        beta[j] = b
        if j == K - 1:
            break
        if b <= tau * scale:
            k_eff = j + 1
            break
        q_prev, q, b_prev = q, w / b, b
    return alpha[:k_eff], beta[:k_eff - 1], Q[:k_eff], beta[k_eff - 1]


def gauss_rule(alpha, beta, vectors=False):
    """Nodes theta_k (eigenvalues of T) and weights w_k = (first eigenvector component)^2."""
    if alpha.size == 1:
        theta = alpha.copy()
        S = np.ones((1, 1))
    else:
        theta, S = scipy.linalg.eigh_tridiagonal(alpha, beta)
    w = S[0, :] ** 2
    if vectors:
        return theta, w, S
    return theta, w


def node_rule(prob, node, **overrides):
    """(theta, w, K_eff) of one node."""
    H = NodeHamiltonian(prob, node, **overrides)
    K = int(prob.depth[node])
    alpha, beta, _, _ = lanczos(H.apply, H.start_vector(), K, H.scale)
    theta, w = gauss_rule(alpha, beta)
    return theta, w, alpha.size


def rho_quadrature(prob, nodes=None, mu=None, kT=None):
    """rho_q = 2 h^-3 sum_k w_k g(theta_k) for every node (or the listed ones).
    Returns (rho, k_eff)."""
    mu = prob.mu if mu is None else mu
    kT = prob.kT if kT is None else kT
    nodes = range(prob.n_nodes) if nodes is None else nodes
    rho, keff = [], []
    for q in nodes:
        theta, w, k = node_rule(prob, q)
        rho.append(2.0 / prob.h ** 3 * float(np.sum(w * fermi(theta, mu, kT))))
        keff.append(k)
    return np.array(rho), np.array(keff, dtype=np.int32)


def band_energy(prob, kind=FREE, nodes=None, mu=None, kT=None, **overrides):
    """Per-node e_q = 2 sum_k w_k F(theta_k) and Omega = sum_q n_q e_q."""
    mu = prob.mu if mu is None else mu
    kT = prob.kT if kT is None else kT
    nodes = list(range(prob.n_nodes)) if nodes is None else list(nodes)
    e = []
    for q in nodes:
        theta, w, _ = node_rule(prob, q, **overrides)
        e.append(2.0 * float(np.sum(w * integrand(theta, mu, kT, kind))))
    e = np.array(e)
    return e, float(np.sum(prob.weight[nodes] * e))


# --------------------------------------------------------------------------------------
# Adjoint of Omega (reverse mode through the exact-arithmetic Lanczos recurrence)
# --------------------------------------------------------------------------------------
def tbar_from_rule(theta, S, mu, kT, kind):
    """Adjoint of e = 2 e_1^T F(T) e_1 with respect to a symmetric T:
    Tbar = 2 S (D o s1 s1^T) S^T (Daleckii-Krein), D the divided differences of F."""
    s1 = S[0, :]
    D = divided_differences(theta, mu, kT, kind)
    return 2.0 * S @ (D * np.outer(s1, s1)) @ S.T


def node_backward(prob, node, kind, scale, **overrides):
    """Gradient of scale * e_node.  Returns (H, vbar over cube points, Ebar per
    projector column, Rbar_nl per projector atom (n_atoms_local, 3))."""
    H = NodeHamiltonian(prob, node, **overrides)
    K = int(prob.depth[node])
    alpha, beta, Q, _ = lanczos(H.apply, H.start_vector(), K, H.scale)
    Ke = alpha.size
    theta, w, S = gauss_rule(alpha, beta, vectors=True)
    Tb = scale * tbar_from_rule(theta, S, prob.mu, prob.kT, kind)
    abar = np.diag(Tb).copy()
    bbar = np.array([2.0 * Tb[j, j + 1] for j in range(Ke - 1)])
    n = Q.shape[1]
    qbar = np.zeros((Ke, n))
    vbar = np.zeros(n)
    pairs = []                       # (u_bar_j, q_j) for the projector adjoints
    for j in range(Ke - 1, -1, -1):
        qj = Q[j]
        uj = H.apply(qj)
        if j < Ke - 1:
            qn = Q[j + 1]
            bb = bbar[j] - float(qbar[j + 1] @ qn) / beta[j]
            rbar = qbar[j + 1] / beta[j] + bb * qn
        else:
            rbar = np.zeros(n)
        ahat = abar[j] - float(rbar @ qj)
        ubar = rbar + ahat * qj
        qbar[j] += -alpha[j] * rbar + ahat * uj + H.apply(ubar)
        if j > 0:
            qbar[j - 1] += -beta[j - 1] * rbar
            bbar[j - 1] -= float(rbar @ Q[j - 1])
        vbar += ubar * qj
        pairs.append((ubar, qj))
    Ebar = None
    Rbar = None
    if H.chi is not None:
        h3 = H.h ** 3
        ncol = H.chi.shape[1]
        Ebar = np.zeros(ncol)
        Rbar = np.zeros((len(H.proj_atoms), 3))
        for ub, qj in pairs:
            cu = H.chi.T @ ub
            cq = H.chi.T @ qj
            Ebar += h3 * cu * cq
            for a in range(3):
                du = H.dchi[a].T @ ub
                dq = H.dchi[a].T @ qj
                # d chi / d R = - d chi / d d
                contrib = -h3 * H.E_cols * (du * cq + cu * dq)
                Rbar[:, a] += contrib.reshape(-1, 4).sum(axis=1)
    return H, vbar, Ebar, Rbar


def band_energy_backward(prob, kind=FREE, grad_omega=1.0, nodes=None):
    """dOmega/dV on the global grid (z, y, x), dOmega/dE (M, 4) and the nonlocal
    part of dOmega/dR (M, 3)."""
    nodes = list(range(prob.n_nodes)) if nodes is None else list(nodes)
    nz, ny, nx = prob.n[2], prob.n[1], prob.n[0]
    dV = np.zeros((nz, ny, nx))
    M = prob.atoms.shape[0]
    dE = np.zeros((M, 4))
    dR = np.zeros((M, 3))
    for q in nodes:
        H, vbar, Ebar, Rbar = node_backward(prob, q, kind, grad_omega * prob.weight[q])
        cube = vbar.reshape(H.shape)
        dV[np.ix_(H.gz, H.gy, H.gx)] += cube
        if Ebar is not None:
            for i, J in enumerate(H.proj_atoms):
                dE[J] += Ebar[4 * i:4 * i + 4]
                dR[J] += Rbar[i]
    return dV, dE, dR


def vloc_position_gradient(dV, n, h, atoms, depth, sigma, cutoff):
    """sum_x dV(x) dV_loc(x)/dR_J for the Gaussian local potential
    V(x) = depth sum_J sum_images exp(-|x - R_J - L m|^2 / (2 sigma^2)) (terms with
    distance <= cutoff*sigma), so dV/dR_J = depth exp(..) (x - R_J - L m)/sigma^2."""
    nx, ny, nz = n
    rcut = cutoff * sigma
    wdt = int(math.ceil(rcut / h)) + 1
    offs = np.arange(-wdt, wdt + 1)
    out = np.zeros((atoms.shape[0], 3))
    for J in range(atoms.shape[0]):
        g = np.floor(atoms[J] / h).astype(np.int64)
        ix, iy, iz = g[0] + offs, g[1] + offs, g[2] + offs
        dx = (ix * h - atoms[J, 0])[None, None, :]
        dy = (iy * h - atoms[J, 1])[None, :, None]
        dz = (iz * h - atoms[J, 2])[:, None, None]
        r2 = dx * dx + dy * dy + dz * dz
        e = np.where(r2 <= rcut * rcut, np.exp(-r2 / (2.0 * sigma * sigma)), 0.0)
        sub = dV[np.ix_(np.mod(iz, nz), np.mod(iy, ny), np.mod(ix, nx))]
        base = depth * e * sub / (sigma * sigma)
        out[J, 0] = np.sum(base * dx)
        out[J, 1] = np.sum(base * dy)
        out[J, 2] = np.sum(base * dz)
    return out


# --------------------------------------------------------------------------------------
# Fermi level (Eq. Eqn:LSSGQ:Fermi_level:GQ, coarse-grained with the node weights of
# Eq. eq:free_cg)
# --------------------------------------------------------------------------------------
def electron_count(theta, w, weight, mu, kT):
    """N(mu) = 2 sum_q n_q sum_k w_k^q g(theta_k^q; mu) for rules theta, w [Nq, K] (padding
    entries carry w = 0) and node weights n_q."""
    theta = np.asarray(theta, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    occ = fermi(theta.ravel(), mu, kT).reshape(theta.shape)
    return 2.0 * float(np.sum(np.asarray(weight, dtype=np.float64)[:, None] * w * occ))


def fermi_level(theta, w, weight, n_electrons, kT, xtol=1e-13):
    """The mu with N(mu) = n_electrons (N increases strictly with mu), by Brent's method on
    a bracket that spans every node of every rule by 60 kT."""
    theta = np.asarray(theta, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    live = w > 0
    total = 2.0 * float(np.sum(np.asarray(weight, dtype=np.float64)[:, None] * w))
    if not (0.0 < n_electrons < total):
        raise ValueError("n_electrons must lie strictly between 0 and 2 sum_q n_q sum_k w_k")
    lo = float(theta[live].min()) - 60.0 * kT
    hi = float(theta[live].max()) + 60.0 * kT
    f = lambda mu: electron_count(theta, w, weight, mu, kT) - n_electrons
    return float(scipy.optimize.brentq(f, lo, hi, xtol=xtol, rtol=4.0 * np.finfo(float).eps,
                                       maxiter=500))


# --------------------------------------------------------------------------------------
# Cluster-sampled energy (Eq. eq:free_cg with the cluster averages of
# Eq. eq:free_cg_sampling)
# --------------------------------------------------------------------------------------
def cluster_members(n, h, center, radius):
    """Grid points (linear indices, ascending) within distance `radius` of grid point
    `center` on the periodic grid n (minimum-image distance), by brute force.  The
    squared distance in grid units is an integer; it is compared with (radius/h)^2
    widened by a relative 1e-9, so a radius equal to a lattice distance takes in that
    shell whatever the rounding of radius itself."""
    nx, ny, nz = n
    lim = (radius / h) ** 2 * (1.0 + 1e-9)
    cx, cy, cz = center % nx, (center // nx) % ny, center // (nx * ny)
    out = []
    for iz in range(nz):
        dz = min(abs(iz - cz), nz - abs(iz - cz))
        for iy in range(ny):
            dy = min(abs(iy - cy), ny - abs(iy - cy))
            for ix in range(nx):
                dx = min(abs(ix - cx), nx - abs(ix - cx))
                if dx * dx + dy * dy + dz * dz <= lim:
                    out.append(ix + nx * (iy + ny * iz))
    return np.array(sorted(out), dtype=np.int64)


def cluster_energy(e_of_point, n, h, esp_centers, esp_weights, radius):
    """E = sum_q n_q Fbar_q with Fbar_q the mean of the per-point energies e_p over the
    cluster of grid points within `radius` of ESP q.  e_of_point maps a grid index to e_p.
    Returns (E, Fbar)."""
    fbar = []
    for c in esp_centers:
        members = cluster_members(n, h, int(c), radius)
        fbar.append(float(np.mean([e_of_point(int(p)) for p in members])))
    fbar = np.array(fbar)
    return float(np.sum(np.asarray(esp_weights, dtype=np.float64) * fbar)), fbar


# --------------------------------------------------------------------------------------
# Predictor + corrector reconstruction on the fine grid (Eq. eq:pc with the FE
# interpolation of the correctors, Eq. phi_approx_scheme)
# --------------------------------------------------------------------------------------
def esp_coords(n, esp_center):
    """Unwrapped integer grid coordinates (M, 3) of the ESPs (linear grid indices)."""
    nx, ny, _ = n
    c = np.asarray(esp_center, dtype=np.int64)
    return np.stack([c % nx, (c // nx) % ny, c // (nx * ny)], axis=1)


def _det3(a, b, c):
    """Exact integer determinant of the rows a, b, c (arrays (..., 3) of int64)."""
    return (a[..., 0] * (b[..., 1] * c[..., 2] - b[..., 2] * c[..., 1])
            - a[..., 1] * (b[..., 0] * c[..., 2] - b[..., 2] * c[..., 0])
            + a[..., 2] * (b[..., 0] * c[..., 1] - b[..., 1] * c[..., 0]))


def fe_locate(n, esp_center, tets, points):
    """For every integer point (P, 3), the lowest-numbered tetrahedron of the ESP mesh
    that contains it (closed: faces, edges and vertices included), -1 if none.

    A point x lies in the tetrahedron (v0, v1, v2, v3) when, with D the signed volume
    det[v1-v0, v2-v0, v3-v0], each of the four volumes D_i(x) obtained by putting x in
    place of vertex i has the sign of D or is zero.  Tetrahedra of zero volume hold no
    interior and are skipped.  D_i is affine in x; its coefficients are read off the
    determinant itself at x = 0 and x = e_x, e_y, e_z (exact integers), and D_i at all
    points is then one matrix product per tetrahedron block, exact in FP64 because every
    value stays below 2^53 for grid coordinates below 2^16.  Brute force over all
    tetrahedra."""
    X = esp_coords(n, esp_center)
    V = X[np.asarray(tets, dtype=np.int64)]                  # (T, 4, 3)
    D = _det3(V[:, 1] - V[:, 0], V[:, 2] - V[:, 0], V[:, 3] - V[:, 0])
    good = D != 0
    sgn = np.sign(D)

    def volume_with(i, x):                                    # D_i at one point x (3,)
        W = [V[:, j] if j != i else np.broadcast_to(x, V[:, 0].shape) for j in range(4)]
        return _det3(W[1] - W[0], W[2] - W[0], W[3] - W[0])

    coef = np.zeros((4, V.shape[0], 4), dtype=np.int64)       # (i, T, [c0, cx, cy, cz])
    for i in range(4):
        c0 = volume_with(i, np.zeros(3, dtype=np.int64))
        coef[i, :, 0] = c0
        for a in range(3):
            e = np.zeros(3, dtype=np.int64)
            e[a] = 1
            coef[i, :, 1 + a] = volume_with(i, e) - c0
    coef = coef * sgn[None, :, None]                          # orient: inside <=> all >= 0
    pts = np.asarray(points, dtype=np.int64)
    P1 = np.hstack([np.ones((pts.shape[0], 1)), pts.astype(np.float64)])   # (P, 4)
    out = np.full(pts.shape[0], -1, dtype=np.int64)
    step = max(1, (1 << 22) // max(1, pts.shape[0]))
    for t0 in range(0, V.shape[0], step):
        inside = np.broadcast_to(good[None, t0:t0 + step], (pts.shape[0], min(step, V.shape[0] - t0))).copy()
        for i in range(4):
            inside &= (P1 @ coef[i, t0:t0 + step].T.astype(np.float64)) >= 0.0
        hit = inside.any(axis=1) & (out < 0)
        out[hit] = t0 + inside[hit].argmax(axis=1)
    return out


def fe_reconstruct(n, esp_center, tets, esp_values, predictor, points=None):
    """Fields on the fine grid from their predictors and the ESP values (Eq. eq:pc):
    f_p = f0_p + sum_q gamma(r_p, r_q) fc_q with the corrector fc_q = f_q - f0(r_q) at
    the ESPs and gamma the linear (barycentric) shape functions of the tetrahedron that
    holds r_p (Eq. phi_approx_scheme); points outside every tetrahedron keep the
    predictor.  esp_values (F, M), predictor (F, nz, ny, nx) or (F, npts).  Returns the
    fields at `points` (linear grid indices; default every grid point), shape (F, P).
    The barycentric coordinates solve the 4x4 system [v_i; 1] lam = [x; 1]."""
    nx, ny, nz = n
    pred = np.asarray(predictor, dtype=np.float64).reshape(len(esp_values), -1)
    vals = np.asarray(esp_values, dtype=np.float64)
    idx = np.arange(nx * ny * nz) if points is None else np.asarray(points, dtype=np.int64)
    xyz = np.stack([idx % nx, (idx // nx) % ny, idx // (nx * ny)], axis=1)
    loc = fe_locate(n, esp_center, tets, xyz)
    X = esp_coords(n, esp_center).astype(np.float64)
    corr = vals - pred[:, np.asarray(esp_center, dtype=np.int64)]   # (F, M)
    out = pred[:, idx].copy()
    k = np.nonzero(loc >= 0)[0]
    if k.size:
        T = np.asarray(tets, dtype=np.int64)[loc[k]]                # (P, 4)
        A = np.concatenate([np.transpose(X[T], (0, 2, 1)), np.ones((k.size, 1, 4))], axis=1)
        rhs = np.hstack([xyz[k].astype(np.float64), np.ones((k.size, 1))])
        lam = np.linalg.solve(A, rhs[:, :, None])[:, :, 0]          # (P, 4)
        out[:, k] += np.einsum("fpi,pi->fp", corr[:, T], lam)
    return out


# --------------------------------------------------------------------------------------
# Self-consistency ingredients: the LDA exchange-correlation potential (Eq. eq:xc) and the
# electrostatic potential of the periodic Poisson problem (Eq. eq:poisson)
# --------------------------------------------------------------------------------------
# Perdew-Wang (1992) parametrisation of the unpolarised correlation energy per electron
# (Hartree):  eps_c(rs) = -2A (1 + a1 rs) ln(1 + 1 / (2A (b1 rs^1/2 + b2 rs + b3 rs^3/2 + b4 rs^2)))
PW92_A, PW92_A1 = 0.031091, 0.21370
PW92_B = (7.5957, 3.5876, 1.6382, 0.49294)


def pw92_correlation(rs):
    """(eps_c, d eps_c / d rs) of the Perdew-Wang form above, rs > 0 (array)."""
    rs = np.asarray(rs, dtype=np.float64)
    b1, b2, b3, b4 = PW92_B
    sq = np.sqrt(rs)
    Q = 2.0 * PW92_A * (b1 * sq + b2 * rs + b3 * rs * sq + b4 * rs * rs)
    dQ = 2.0 * PW92_A * (0.5 * b1 / sq + b2 + 1.5 * b3 * sq + 2.0 * b4 * rs)
    L = np.log1p(1.0 / Q)
    eps = -2.0 * PW92_A * (1.0 + PW92_A1 * rs) * L
    deps = -2.0 * PW92_A * PW92_A1 * L + 2.0 * PW92_A * (1.0 + PW92_A1 * rs) * (dQ / Q) / (Q + 1.0)
    return eps, deps


def lda_xc(rho):
    """LDA exchange-correlation energy per volume e_xc(rho) = -3/4 (3/pi)^(1/3) rho^(4/3)
    + rho eps_c(rho) and its potential u = d e_xc / d rho (Eq. eq:xc), elementwise; zero where
    rho <= 0.  The correlation part is the Perdew-Wang form in the Wigner-Seitz radius
    rs = (3 / (4 pi rho))^(1/3); its potential is eps_c - rs/3 d eps_c/d rs."""
    rho = np.asarray(rho, dtype=np.float64)
    e = np.zeros_like(rho)
    u = np.zeros_like(rho)
    pos = rho > 0.0
    r = rho[pos]
    cx = (3.0 / math.pi) ** (1.0 / 3.0)
    ex = -0.75 * cx * r ** (4.0 / 3.0)
    ux = -cx * r ** (1.0 / 3.0)
    rs = (3.0 / (4.0 * math.pi * r)) ** (1.0 / 3.0)
    ec, dec = pw92_correlation(rs)
    e[pos] = ex + r * ec
    u[pos] = ux + ec - rs / 3.0 * dec
    return e, u


def fd_laplacian_symbol(n, h):
    """Eigenvalues of the periodic sixth-order FD Laplacian on the grid n (per-axis sums),
    (nz, ny, nx): sum over axes of (w0 + 2 sum_m w_m cos(2 pi m k / n_a)) / h^2."""
    nx, ny, nz = n
    def axis(na):
        k = np.arange(na)
        return sum((FD2_WEIGHTS[0] if m == 0 else 2.0 * FD2_WEIGHTS[m] * np.cos(2.0 * math.pi * m * k / na))
                   for m in range(4)) / (h * h)
    return axis(nz)[:, None, None] + axis(ny)[None, :, None] + axis(nx)[None, None, :]


def poisson_periodic(source, h):
    """phi with -(1/4 pi) Lap_6 phi = s - mean(s) on the periodic grid (Eq. eq:poisson, the
    FD Laplacian of the Hamiltonian), mean(phi) = 0; by FFT, dividing by the FD symbol.
    source (nz, ny, nx).  Returns (phi, mean(s))."""
    s = np.asarray(source, dtype=np.float64)
    nz, ny, nx = s.shape
    lam = fd_laplacian_symbol((nx, ny, nz), h)
    sk = np.fft.fftn(s)
    # every FD eigenvalue but the k = 0 one is strictly negative; the k = 0 mode (the mean)
    # is dropped by its index (its computed eigenvalue is a rounding residue, not 0)
    lam[0, 0, 0] = 1.0
    phik = -4.0 * math.pi * sk / lam
    phik[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(phik)), float(np.mean(s))


def effective_potential(rho, b, h):
    """V = phi[rho + b] + u(rho): the electrostatic and exchange-correlation parts of the
    Hamiltonian's potential (Eq. Eqn:Hamiltonian) from the electron density rho and the
    nuclear charge density b on the grid.  Returns (V, e_xc, phi, mean(rho + b))."""
    phi, mean = poisson_periodic(np.asarray(rho) + np.asarray(b), h)
    e, u = lda_xc(rho)
    return phi + u, e, phi, mean


# --------------------------------------------------------------------------------------
# Error metrics
# --------------------------------------------------------------------------------------
def normwise_rel_err(got, ref):
    """||got - ref||_inf / ||ref||_inf."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.max(np.abs(ref))
    return float(np.max(np.abs(got - ref)) / den) if den > 0 else float(np.max(np.abs(got - ref)))
