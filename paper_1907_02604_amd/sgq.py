"""ctypes binding of libsgq.so (argument marshalling only).

Every compute step runs in the HIP library; this module passes device pointers of
torch tensors and the current HIP stream to the C ABI declared in include/sgq.h.
Importing it loads the in-tree library and fails loudly when it is missing.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("SGQ_LIBRARY") or os.path.join(_HERE, "libsgq.so")

SGQ_OK, SGQ_EINVAL, SGQ_ENOMEM, SGQ_EHIP, SGQ_EPLAN, SGQ_ENONFINITE, SGQ_ELIMIT = 0, -1, -2, -3, -4, -5, -6
SGQ_ERANGE, SGQ_EINDEX = -7, -8
SGQ_FP64, SGQ_FP32 = 0, 1
SGQ_BAND, SGQ_FREE, SGQ_GRAND = 0, 1, 2
SGQ_SCHEDULE_BATCHED, SGQ_SCHEDULE_PLAIN = 0, 1

EXPORTED = ("sgq_plan_create", "sgq_plan_destroy", "rho_quadrature", "band_energy",
            "band_energy_backward", "sgq_vloc_gaussian_backward", "sgq_plan_status",
            "sgq_last_error", "sgq_validate", "sgq_gauss_rule_host", "sgq_plan_set_schedule",
            "sgq_plan_set_graph", "sgq_plan_autotune", "sgq_fermi_level", "sgq_cluster_build",
            "sgq_cluster_energy", "sgq_fe_mesh_create", "sgq_fe_mesh_destroy",
            "sgq_fe_reconstruct", "sgq_fe_mesh_location", "sgq_fe_mesh_info", "sgq_lda_xc",
            "sgq_potential_create", "sgq_potential_destroy", "sgq_poisson",
            "sgq_effective_potential", "sgq_plan_set_retain", "sgq_plan_prepare_backward",
            "sgq_fermi_level_noalloc")


class SgqError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sgq error {code}: {msg}")
        self.code = code


class Problem(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32 * 3), ("h", ctypes.c_double), ("n_atoms", ctypes.c_int32),
                ("n_proj", ctypes.c_int32), ("proj_rc", ctypes.c_double),
                ("proj_rg", ctypes.c_double), ("n_nodes", ctypes.c_int32),
                ("precision", ctypes.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_1907_02604_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, V = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, None
    sig = {
        "sgq_plan_create": (I, [ctypes.POINTER(Problem), P, P, P, ctypes.POINTER(P)]),
        "sgq_plan_destroy": (I, [P]),
        "rho_quadrature": (I, [P, P, P, P, D, D, P, P, P, P]),
        "band_energy": (I, [P, P, P, P, P, D, D, I, P, P, P]),
        "band_energy_backward": (I, [P, P, P, P, P, D, D, I, P, P, P, P, P]),
        "sgq_vloc_gaussian_backward": (I, [P, P, P, D, D, D, P, P]),
        "sgq_plan_status": (I, [P, ctypes.POINTER(ctypes.c_int32)]),
        "sgq_last_error": (ctypes.c_char_p, []),
        "sgq_validate": (I, [ctypes.POINTER(Problem), P, P, P]),
        "sgq_gauss_rule_host": (I, [P, P, I, P, P]),
        "sgq_plan_set_schedule": (I, [P, I]),
        "sgq_plan_set_graph": (I, [P, I]),
        "sgq_plan_set_retain": (I, [P, I, ctypes.c_int64, P]),
        "sgq_plan_prepare_backward": (I, [P]),
        "sgq_fermi_level": (I, [P, P, P, D, D, D, P, P]),
        "sgq_fermi_level_noalloc": (I, [P, P, ctypes.c_int32, ctypes.c_int32, D, D, D, P, P, P]),
        "sgq_plan_autotune": (I, [P, P, P, P, D, D, I, P, ctypes.POINTER(ctypes.c_int32)]),
        "sgq_cluster_build": (I, [P, D, P, ctypes.c_int32, D, P, ctypes.c_int64, ctypes.c_int64,
                                  P, P, P, P, P, P, P]),
        "sgq_cluster_energy": (I, [P, P, P, P, ctypes.c_int64, ctypes.c_int32, P, P, P, P]),
        "sgq_fe_mesh_create": (I, [P, P, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32,
                                   ctypes.POINTER(P)]),
        "sgq_fe_mesh_destroy": (I, [P]),
        "sgq_fe_reconstruct": (I, [P, ctypes.c_int32, P, P, P, P]),
        "sgq_fe_mesh_location": (I, [P, P, P]),
        "sgq_fe_mesh_info": (I, [P, P]),
        "sgq_lda_xc": (I, [P, ctypes.c_int64, P, P, P]),
        "sgq_potential_create": (I, [P, D, ctypes.POINTER(P)]),
        "sgq_potential_destroy": (I, [P]),
        "sgq_poisson": (I, [P, P, P, P, P]),
        "sgq_effective_potential": (I, [P, P, P, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    del V
    return lib


_lib = _load()


def lib():
    return _lib


def _check(code):
    if code != SGQ_OK:
        raise SgqError(code, _lib.sgq_last_error().decode())


def _ptr(t):
    """Device (or host numpy) pointer of a contiguous array, None for None."""
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        assert t.flags.c_contiguous
        return t.ctypes.data
    assert t.is_contiguous(), "tensors passed to libsgq must be contiguous"
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


def make_problem_struct(n, h, n_atoms, n_proj, n_nodes, precision, proj_rc=1.5, proj_rg=0.5):
    p = Problem()
    p.n[0], p.n[1], p.n[2] = int(n[0]), int(n[1]), int(n[2])
    p.h = float(h)
    p.n_atoms = int(n_atoms)
    p.n_proj = int(n_proj)
    p.proj_rc = float(proj_rc)
    p.proj_rg = float(proj_rg)
    p.n_nodes = int(n_nodes)
    p.precision = int(precision)
    return p


def validate(n, h, n_atoms, n_proj, centers, half_width, depth, precision, proj_rc=1.5, proj_rg=0.5):
    """Host-only argument check (sgq_validate); returns the status code."""
    c = np.ascontiguousarray(centers, dtype=np.int64)
    hw = np.ascontiguousarray(half_width, dtype=np.int32)
    d = np.ascontiguousarray(depth, dtype=np.int32)
    prob = make_problem_struct(n, h, n_atoms, n_proj, c.size, precision, proj_rc, proj_rg)
    return _lib.sgq_validate(ctypes.byref(prob), c.ctypes.data, hw.ctypes.data, d.ctypes.data)


def gauss_rule_host(alpha, beta):
    """(theta ascending, weights) of the tridiagonal (alpha, beta) via the library's host solver."""
    a = np.ascontiguousarray(alpha, dtype=np.float64)
    b = np.ascontiguousarray(beta, dtype=np.float64)
    K = a.size
    th = np.zeros(K)
    w = np.zeros(K)
    _check(_lib.sgq_gauss_rule_host(a.ctypes.data, b.ctypes.data if b.size else None, K,
                                    th.ctypes.data, w.ctypes.data))
    return th, w


class Plan:
    """A plan for a fixed grid and node set (sgq_plan_create)."""

    def __init__(self, n, h, n_atoms, n_proj, centers, half_width, depth, precision,
                 proj_rc=1.5, proj_rg=0.5):
        c = np.ascontiguousarray(centers, dtype=np.int64)
        hw = np.ascontiguousarray(half_width, dtype=np.int32)
        d = np.ascontiguousarray(depth, dtype=np.int32)
        self.n = tuple(int(v) for v in n)
        self.n_nodes = int(c.size)
        self.n_atoms = int(n_atoms)
        self.n_proj = int(n_proj)
        self.kmax = int(d.max()) if d.size else 1
        self.precision = int(precision)
        prob = make_problem_struct(n, h, n_atoms, n_proj, c.size, precision, proj_rc, proj_rg)
        handle = ctypes.c_void_p()
        _check(_lib.sgq_plan_create(ctypes.byref(prob), c.ctypes.data, hw.ctypes.data,
                                    d.ctypes.data, ctypes.byref(handle)))
        self._h = handle

    @classmethod
    def from_problem(cls, prob):
        """Plan for a ``synth.Problem``."""
        prec = SGQ_FP64 if prob.precision == "f64" else SGQ_FP32
        return cls(prob.n, prob.h, prob.atoms.shape[0], prob.n_proj, prob.centers,
                   prob.half_width, prob.depth, prec)

    @property
    def handle(self):
        return self._h

    def set_schedule(self, schedule):
        """SGQ_SCHEDULE_BATCHED (default) or SGQ_SCHEDULE_PLAIN (per-node baseline)."""
        _check(_lib.sgq_plan_set_schedule(self._h, int(schedule)))

    def set_retain(self, enable, max_bytes=0):
        """sgq_plan_set_retain: keep the forward bases for the next backward call, of every
        node (max_bytes 0) or of the costliest nodes that fit in max_bytes.  Returns the
        number of nodes retained."""
        n = ctypes.c_int64(0)
        _check(_lib.sgq_plan_set_retain(self._h, 1 if enable else 0, int(max_bytes),
                                        ctypes.byref(n)))
        return n.value

    def prepare_backward(self):
        """sgq_plan_prepare_backward: allocate the backward workspace (synchronous; a no-op
        once done)."""
        _check(_lib.sgq_plan_prepare_backward(self._h))

    def set_graph(self, enable):
        """Capture and replay the forward launches as a HIP graph (default on)."""
        _check(_lib.sgq_plan_set_graph(self._h, int(bool(enable))))

    def autotune(self, v_loc, atom_R, proj_E, mu, kT, sample_nodes=2048, stream=None):
        """Pick the launch shape of the forward kernel by timing candidates on a sample of
        this plan's nodes (sgq_plan_autotune); returns (lanes per node, workgroups per CU)."""
        out = (ctypes.c_int32 * 2)()
        _check(_lib.sgq_plan_autotune(self._h, _ptr(v_loc), _ptr(atom_R), _ptr(proj_E),
                                      float(mu), float(kT), int(sample_nodes),
                                      _stream(stream), out))
        return int(out[0]), int(out[1])

    def status(self):
        st = ctypes.c_int32(0)
        _check(_lib.sgq_plan_status(self._h, ctypes.byref(st)))
        return int(st.value)

    def close(self):
        if self._h is not None and self._h.value:
            _lib.sgq_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rho_quadrature(plan, v_loc, atom_R, proj_E, mu, kT, rho, theta_w=None, k_eff=None, stream=None):
    _check(_lib.rho_quadrature(plan.handle, _ptr(v_loc), _ptr(atom_R), _ptr(proj_E), float(mu),
                               float(kT), _ptr(rho), _ptr(theta_w), _ptr(k_eff), _stream(stream)))


def band_energy(plan, v_loc, atom_R, proj_E, node_weight, mu, kT, integrand, e_node, omega,
                stream=None):
    _check(_lib.band_energy(plan.handle, _ptr(v_loc), _ptr(atom_R), _ptr(proj_E), _ptr(node_weight),
                            float(mu), float(kT), int(integrand), _ptr(e_node), _ptr(omega),
                            _stream(stream)))


def band_energy_backward(plan, v_loc, atom_R, proj_E, node_weight, mu, kT, integrand, grad_omega,
                         dV, dR_nl, dE=None, stream=None):
    _check(_lib.band_energy_backward(plan.handle, _ptr(v_loc), _ptr(atom_R), _ptr(proj_E),
                                     _ptr(node_weight), float(mu), float(kT), int(integrand),
                                     _ptr(grad_omega), _ptr(dV), _ptr(dR_nl), _ptr(dE),
                                     _stream(stream)))


def fermi_level(plan, theta_w, node_weight, n_electrons, kT, result, tol=1e-12, stream=None):
    """sgq_fermi_level: result (device, 3 doubles) <- mu, N(mu), steps."""
    _check(_lib.sgq_fermi_level(plan.handle, _ptr(theta_w), _ptr(node_weight),
                                float(n_electrons), float(kT), float(tol), _ptr(result),
                                _stream(stream)))


def fermi_level_noalloc(theta_w, node_weight, n_nodes, kmax, n_electrons, kT, result, status,
                        tol=1e-12, stream=None):
    """sgq_fermi_level_noalloc: result (device, 3 doubles) <- mu, N(mu), steps; status
    (device int32) <- the solve's sgq_status.  Returns the call's own status code (host
    argument checks), without raising."""
    return _lib.sgq_fermi_level_noalloc(_ptr(theta_w), _ptr(node_weight), int(n_nodes), int(kmax),
                                        float(n_electrons), float(kT), float(tol), _ptr(result),
                                        _ptr(status), _stream(stream))


def cluster_build(n, h, esp_center, radius, esp_weight=None):
    """sgq_cluster_build on host arrays.  Returns a dict of numpy arrays: node_center,
    node_esp, member_offset, member_node and (with esp_weight) node_weight."""
    dims = np.ascontiguousarray([int(v) for v in n], dtype=np.int32)
    c = np.ascontiguousarray(esp_center, dtype=np.int64)
    w = None if esp_weight is None else np.ascontiguousarray(esp_weight, dtype=np.float64)
    nn, nm = ctypes.c_int64(0), ctypes.c_int64(0)
    args = (dims.ctypes.data, float(h), c.ctypes.data if c.size else None, int(c.size),
            float(radius), _ptr(w))
    _check(_lib.sgq_cluster_build(*args, 0, 0, None, None, None, None, None,
                                  ctypes.byref(nn), ctypes.byref(nm)))
    out = {"node_center": np.zeros(nn.value, np.int64), "node_esp": np.zeros(nn.value, np.int32),
           "member_offset": np.zeros(c.size + 1, np.int64),
           "member_node": np.zeros(nm.value, np.int32)}
    if w is not None:
        out["node_weight"] = np.zeros(nn.value, np.float64)
    _check(_lib.sgq_cluster_build(*args, nn.value, nm.value, out["node_center"].ctypes.data,
                                  out["node_esp"].ctypes.data, _ptr(out.get("node_weight")),
                                  out["member_offset"].ctypes.data, out["member_node"].ctypes.data,
                                  ctypes.byref(nn), ctypes.byref(nm)))
    return out


def torch_int64():
    import torch
    return torch.int64


def torch_int32():
    import torch
    return torch.int32


def cluster_energy(plan, e_node, member_offset, member_node, esp_weight, fbar, energy=None,
                   stream=None):
    """sgq_cluster_energy: fbar[q] <- mean of e_node over cluster q; energy <- sum n_q fbar_q."""
    n_esp = int(member_offset.numel()) - 1
    assert member_offset.dtype == torch_int64() and member_node.dtype == torch_int32()
    _check(_lib.sgq_cluster_energy(plan.handle, _ptr(e_node), _ptr(member_offset),
                                   _ptr(member_node), int(member_node.numel()), n_esp,
                                   _ptr(esp_weight), _ptr(fbar), _ptr(energy), _stream(stream)))


class FeMesh:
    """sgq_fe_mesh: a tetrahedral mesh over ESPs on the grid and the location of every grid
    point in it (built on the current device at creation)."""

    def __init__(self, n, esp_center, tets, max_fields=2):
        dims = np.ascontiguousarray([int(v) for v in n], dtype=np.int32)
        c = np.ascontiguousarray(esp_center, dtype=np.int64)
        t = np.ascontiguousarray(tets, dtype=np.int32).reshape(-1, 4)
        self.n = tuple(int(v) for v in n)
        self.n_esp = int(c.size)
        self._h = ctypes.c_void_p()
        _check(_lib.sgq_fe_mesh_create(dims.ctypes.data, c.ctypes.data, int(c.size),
                                       t.ctypes.data if t.size else None, int(t.shape[0]),
                                       int(max_fields), ctypes.byref(self._h)))

    @property
    def handle(self):
        return self._h

    def info(self):
        out = np.zeros(5, np.int64)
        _check(_lib.sgq_fe_mesh_info(self._h, out.ctypes.data))
        return dict(zip(("npts", "n_esp", "n_tets", "kept", "bucket"), out.tolist()))

    def location(self, loc, stream=None):
        _check(_lib.sgq_fe_mesh_location(self._h, _ptr(loc), _stream(stream)))

    def reconstruct(self, esp_values, predictor, out, stream=None):
        """esp_values (F, n_esp), predictor and out (F, npts): contiguous FP64 device tensors."""
        F = int(esp_values.shape[0])
        assert esp_values.numel() == F * self.n_esp
        assert predictor.numel() == out.numel() == F * int(np.prod(self.n))
        _check(_lib.sgq_fe_reconstruct(self._h, F, _ptr(esp_values), _ptr(predictor), _ptr(out),
                                       _stream(stream)))

    def close(self):
        if self._h:
            _lib.sgq_fe_mesh_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def lda_xc(rho, vxc, exc=None, stream=None):
    """sgq_lda_xc on contiguous FP64 device tensors of equal size."""
    _check(_lib.sgq_lda_xc(_ptr(rho), int(rho.numel()), _ptr(exc), _ptr(vxc), _stream(stream)))


class Potential:
    """sgq_potential: the periodic Poisson solver (and effective potential) of a grid."""

    def __init__(self, n, h):
        dims = np.ascontiguousarray([int(v) for v in n], dtype=np.int32)
        self.n = tuple(int(v) for v in n)
        self._h = ctypes.c_void_p()
        _check(_lib.sgq_potential_create(dims.ctypes.data, float(h), ctypes.byref(self._h)))

    def poisson(self, source, phi, mean=None, stream=None):
        _check(_lib.sgq_poisson(self._h, _ptr(source), _ptr(phi), _ptr(mean), _stream(stream)))

    def effective(self, rho, v, b=None, phi=None, exc=None, mean=None, stream=None):
        _check(_lib.sgq_effective_potential(self._h, _ptr(rho), _ptr(b), _ptr(v), _ptr(phi),
                                            _ptr(exc), _ptr(mean), _stream(stream)))

    def close(self):
        if self._h:
            _lib.sgq_potential_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def vloc_gaussian_backward(plan, dV, atom_R, depth, sigma, cutoff_sigmas, dR, stream=None):
    _check(_lib.sgq_vloc_gaussian_backward(plan.handle, _ptr(dV), _ptr(atom_R), float(depth),
                                           float(sigma), float(cutoff_sigmas), _ptr(dR),
                                           _stream(stream)))


# ------------------------------------------------------------------ torch conveniences
def device_inputs(prob, device="cuda"):
    """Device tensors (v_loc, atoms, proj_E, weight) of a ``synth.Problem``."""
    import torch
    v = torch.as_tensor(np.ascontiguousarray(prob.v_loc), dtype=torch.float64, device=device)
    R = torch.as_tensor(np.ascontiguousarray(prob.atoms), dtype=torch.float64, device=device)
    E = torch.as_tensor(np.ascontiguousarray(prob.proj_E), dtype=torch.float64, device=device)
    w = torch.as_tensor(np.ascontiguousarray(prob.weight), dtype=torch.float64, device=device)
    return v, R, E, w


def cluster_problem(prob, esp, radius, esp_weight=None):
    """Node problem of the cluster sampling around the nodes ``esp`` of a ``synth.Problem``.

    Returns (node problem, cluster lists).  The node problem holds the merged cluster
    nodes (sgq_cluster_build), each with the cube half-width and depth of the lowest ESP
    whose cluster holds it and the node weight sum_q n_q / |C_q| (n_q = esp_weight,
    default the ESPs' own node weights)."""
    import dataclasses
    esp = np.asarray(esp, dtype=np.int64)
    w = prob.weight[esp] if esp_weight is None else np.asarray(esp_weight, dtype=np.float64)
    cl = cluster_build(prob.n, prob.h, prob.centers[esp], radius, esp_weight=w)
    src = esp[cl["node_esp"]]
    nodes = dataclasses.replace(prob, centers=cl["node_center"].copy(),
                                half_width=prob.half_width[src].copy(),
                                depth=prob.depth[src].copy(), weight=cl["node_weight"].copy())
    cl["esp_weight"] = w
    return nodes, cl


def rho(prob, plan=None, want_rule=False, device="cuda"):
    """Density at the nodes of a ``synth.Problem``; returns torch tensors."""
    import torch
    plan = plan or Plan.from_problem(prob)
    v, R, E, _ = device_inputs(prob, device)
    out = torch.empty(prob.n_nodes, dtype=torch.float64, device=device)
    tw = torch.zeros(prob.n_nodes * plan.kmax * 2, dtype=torch.float64, device=device) if want_rule else None
    ke = torch.zeros(prob.n_nodes, dtype=torch.int32, device=device)
    rho_quadrature(plan, v, R, E, prob.mu, prob.kT, out, tw, ke)
    if want_rule:
        return out, tw.view(prob.n_nodes, plan.kmax, 2), ke
    return out, ke


def energy(prob, kind=SGQ_FREE, plan=None, device="cuda"):
    """(e_node, Omega) of a ``synth.Problem`` as torch tensors."""
    import torch
    plan = plan or Plan.from_problem(prob)
    v, R, E, w = device_inputs(prob, device)
    e = torch.empty(prob.n_nodes, dtype=torch.float64, device=device)
    om = torch.empty(1, dtype=torch.float64, device=device)
    band_energy(plan, v, R, E, w, prob.mu, prob.kT, kind, e, om)
    return e, om


def energy_backward(prob, kind=SGQ_FREE, grad_omega=1.0, plan=None, device="cuda"):
    """(dV [z,y,x], dR_nl [M,3], dE [M,4]) of Omega for a ``synth.Problem``."""
    import torch
    plan = plan or Plan.from_problem(prob)
    plan.prepare_backward()
    v, R, E, w = device_inputs(prob, device)
    g = torch.full((1,), float(grad_omega), dtype=torch.float64, device=device)
    dV = torch.empty_like(v)
    dR = torch.zeros_like(R)
    dE = torch.zeros_like(E)
    band_energy_backward(plan, v, R, E, w, prob.mu, prob.kT, kind, g, dV, dR, dE)
    return dV, dR, dE


def _autograd():
    import torch

    class BandEnergy(torch.autograd.Function):
        """Omega(V_loc, R, E) = sum_q n_q e_q through libsgq, with the hand-written adjoint.

        forward: band_energy; backward: band_energy_backward (dV, the projector part of
        dR, dE).  When ``vloc_model = (depth, sigma, cutoff_sigmas)`` is given, V_loc is
        taken as that Gaussian function of R and its chain rule is added to dR."""

        @staticmethod
        def forward(ctx, v_loc, atom_R, proj_E, plan, node_weight, mu, kT, integrand, vloc_model):
            e = torch.empty(plan.n_nodes, dtype=torch.float64, device=v_loc.device)
            om = torch.empty(1, dtype=torch.float64, device=v_loc.device)
            v_loc, atom_R, proj_E = v_loc.contiguous(), atom_R.contiguous(), proj_E.contiguous()
            if ctx.needs_input_grad[0] or ctx.needs_input_grad[1] or ctx.needs_input_grad[2]:
                plan.prepare_backward()   # set-up: the backward call itself allocates nothing
            band_energy(plan, v_loc, atom_R, proj_E, node_weight, mu, kT, integrand, e, om)
            ctx.save_for_backward(v_loc, atom_R, proj_E, node_weight)
            ctx.plan, ctx.mu, ctx.kT, ctx.integrand, ctx.vloc_model = plan, mu, kT, integrand, vloc_model
            return om[0]

        @staticmethod
        def backward(ctx, g):
            v_loc, atom_R, proj_E, node_weight = ctx.saved_tensors
            gw = g.reshape(1).to(torch.float64).contiguous()
            dV = torch.empty_like(v_loc)
            dR = torch.zeros_like(atom_R)
            dE = torch.zeros_like(proj_E)
            band_energy_backward(ctx.plan, v_loc, atom_R, proj_E, node_weight, ctx.mu, ctx.kT,
                                 ctx.integrand, gw, dV, dR, dE)
            if ctx.vloc_model is not None:
                depth, sigma, cutoff = ctx.vloc_model
                vloc_gaussian_backward(ctx.plan, dV, atom_R, depth, sigma, cutoff, dR)
            return dV, dR, dE, None, None, None, None, None, None

    return BandEnergy


def band_energy_fn(v_loc, atom_R, proj_E, plan, node_weight, mu, kT, integrand=SGQ_FREE,
                   vloc_model=None):
    """Differentiable Omega (a 0-d tensor) for torch autograd."""
    return _autograd().apply(v_loc, atom_R, proj_E, plan, node_weight, mu, kT, integrand, vloc_model)
