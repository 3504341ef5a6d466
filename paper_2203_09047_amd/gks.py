"""Python binding of the gks C ABI: argument marshalling only.

PyTorch supplies device memory and streams; every step of the solver runs in
the HIP kernels of ``libgks.so``.  The binding fails loudly when the library is
missing or no GPU is present: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgks.so")

GKS_OK, GKS_EINVAL, GKS_EDEVICE, GKS_ESINGULAR, GKS_ENONPHYS, GKS_EMESH = range(6)
FP64, FP32_MIXED = 0, 1
STATUS_NAMES = {0: "OK", 1: "EINVAL", 2: "EDEVICE", 3: "ESINGULAR", 4: "ENONPHYS", 5: "EMESH"}

SYMBOLS = [
    "gks_default_params", "gks_preprocess", "gks_host_mesh_free", "gks_host_mesh_counts", "gks_host_mesh_perm",
    "gks_host_mesh_geometry", "gks_host_mesh_faces", "gks_host_mesh_face_geometry", "gks_mesh_sizes", "gks_init_mesh",
    "gks_destroy_mesh",
    "gks_reset_status", "gks_timestep", "gks_reconstruct", "gks_flux", "gks_residual", "gks_s2o4_step",
    "gks_poll_status", "gks_fallback_count", "gks_gp_flux_batch", "gks_profile", "gks_profile_read", "gks_gp_op_count",
    "gks_gp_flux_host", "gks_gp_flux_vjp_host", "gks_weno_combine_host", "gks_weno_combine_vjp_host",
    "gks_adjoint_work_bytes", "gks_adjoint_step", "gks_kinetic_energy", "gks_last_error", "gks_implicit_step",
    "gks_set_flux_window", "gks_s2o4_step_noalloc",
]
KERNELS = ("timestep", "reconstruct", "flux", "stage1", "stage2", "residual", "flux_adj", "reconstruct_adj",
           "gather_adj", "implicit")


class GksError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


BC_SLIP, BC_NOSLIP, BC_ISOTHERMAL, BC_FARFIELD, BC_EXTRAPOLATE = range(5)


class Boundary(ctypes.Structure):
    """gks_boundary: condition of one box plane (type, wall velocity, wall temperature, free stream)."""

    _fields_ = [("type", ctypes.c_int), ("uw", ctypes.c_double * 3), ("Tw", ctypes.c_double),
                ("far", ctypes.c_double * 5)]


def boundary(type=BC_SLIP, uw=(0.0, 0.0, 0.0), Tw=1.0, far=(1.0, 0.0, 0.0, 0.0, 1.0)) -> Boundary:
    return Boundary(int(type), (ctypes.c_double * 3)(*uw), float(Tw), (ctypes.c_double * 5)(*far))


class Params(ctypes.Structure):
    _fields_ = [
        ("gamma", ctypes.c_double), ("cfl", ctypes.c_double), ("mu", ctypes.c_double), ("Pr", ctypes.c_double),
        ("weno_eps", ctypes.c_double), ("weno_gamma_m", ctypes.c_double), ("weno_p", ctypes.c_double),
        ("tau_eps", ctypes.c_double), ("tau_C", ctypes.c_double), ("viscous", ctypes.c_int),
        ("precision", ctypes.c_int), ("force_linear", ctypes.c_int), ("dt_given", ctypes.c_int),
        ("first_order_fallback", ctypes.c_int), ("fallback_floor", ctypes.c_double), ("smooth_flux", ctypes.c_int),
        ("mu_power", ctypes.c_double), ("T_ref", ctypes.c_double), ("dt_max", ctypes.c_double),
        ("bc", Boundary * 6),
    ]


_lib = None


def load():
    """Load libgks.so (after torch, so that both use torch's HIP runtime)."""
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (loads the HIP runtime the library must share)

        if not os.path.exists(LIB_PATH):
            raise GksError(GKS_EDEVICE, f"{LIB_PATH} is not built; run __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i64, i32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_size_t
        pp = ctypes.POINTER(Params)
        st = ctypes.c_int
        lib.gks_default_params.argtypes = [pp]
        lib.gks_default_params.restype = None
        lib.gks_preprocess.argtypes = [i64, vp, i64, vp, vp, vp, i32, i32, ctypes.POINTER(vp)]
        lib.gks_preprocess.restype = st
        lib.gks_host_mesh_free.argtypes = [vp]
        lib.gks_host_mesh_free.restype = None
        lib.gks_host_mesh_counts.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.gks_host_mesh_counts.restype = st
        lib.gks_host_mesh_perm.argtypes = [vp, vp]
        lib.gks_host_mesh_perm.restype = st
        lib.gks_host_mesh_geometry.argtypes = [vp, vp, vp]
        lib.gks_host_mesh_geometry.restype = st
        lib.gks_host_mesh_faces.argtypes = [vp, vp, vp]
        lib.gks_host_mesh_faces.restype = st
        lib.gks_host_mesh_face_geometry.argtypes = [vp, vp]
        lib.gks_host_mesh_face_geometry.restype = st
        lib.gks_mesh_sizes.argtypes = [vp, i32, ctypes.POINTER(sz), ctypes.POINTER(sz), ctypes.POINTER(sz)]
        lib.gks_mesh_sizes.restype = st
        lib.gks_init_mesh.argtypes = [vp, i32, vp, sz, vp, ctypes.POINTER(vp)]
        lib.gks_init_mesh.restype = st
        lib.gks_destroy_mesh.argtypes = [vp]
        lib.gks_destroy_mesh.restype = None
        lib.gks_reset_status.argtypes = [vp, vp, vp]
        lib.gks_reset_status.restype = st
        lib.gks_timestep.argtypes = [vp, vp, pp, vp, vp, vp]
        lib.gks_timestep.restype = st
        lib.gks_reconstruct.argtypes = [vp, vp, vp, pp, vp, vp]
        lib.gks_reconstruct.restype = st
        lib.gks_flux.argtypes = [vp, vp, vp, vp, vp, pp, vp, vp]
        lib.gks_flux.restype = st
        lib.gks_residual.argtypes = [vp, vp, vp, vp, pp, vp]
        lib.gks_residual.restype = st
        lib.gks_s2o4_step.argtypes = [vp, vp, vp, pp, vp, vp, vp, vp]
        lib.gks_s2o4_step.restype = st
        lib.gks_s2o4_step_noalloc.argtypes = [vp, vp, vp, pp, vp, vp, vp, vp]
        lib.gks_s2o4_step_noalloc.restype = st
        lib.gks_poll_status.argtypes = [vp, vp, vp]
        lib.gks_fallback_count.argtypes = [vp, vp, ctypes.POINTER(i64), vp]
        lib.gks_fallback_count.restype = st
        lib.gks_poll_status.restype = st
        lib.gks_gp_flux_batch.argtypes = [i64, vp, vp, vp, vp, vp, vp, pp, vp]
        lib.gks_gp_flux_batch.restype = st
        lib.gks_set_flux_window.argtypes = [vp, i32]
        lib.gks_set_flux_window.restype = st
        lib.gks_profile.argtypes = [vp, i32]
        lib.gks_profile.restype = st
        lib.gks_profile_read.argtypes = [vp, vp, vp]
        lib.gks_profile_read.restype = st
        lib.gks_gp_op_count.argtypes = [i32, ctypes.c_double, vp, vp, vp, vp]
        lib.gks_gp_op_count.restype = st
        dbl = ctypes.c_double
        lib.gks_gp_flux_host.argtypes = [vp, vp, vp, vp, dbl, pp, vp]
        lib.gks_gp_flux_host.restype = st
        lib.gks_gp_flux_vjp_host.argtypes = [vp, vp, vp, vp, dbl, pp, vp, vp, vp, vp, vp]
        lib.gks_gp_flux_vjp_host.restype = st
        lib.gks_weno_combine_host.argtypes = [vp, vp, vp, i32, dbl, vp, dbl, pp, vp]
        lib.gks_weno_combine_host.restype = st
        lib.gks_weno_combine_vjp_host.argtypes = [vp, vp, vp, i32, dbl, vp, pp, vp, vp, vp, vp]
        lib.gks_weno_combine_vjp_host.restype = st
        lib.gks_adjoint_work_bytes.argtypes = [vp, ctypes.POINTER(sz)]
        lib.gks_adjoint_work_bytes.restype = st
        lib.gks_adjoint_step.argtypes = [vp, vp, vp, vp, vp, vp, pp, vp, vp, vp]
        lib.gks_adjoint_step.restype = st
        lib.gks_implicit_step.argtypes = [vp, vp, vp, dbl, i32, pp, vp, vp]
        lib.gks_implicit_step.restype = st
        lib.gks_kinetic_energy.argtypes = [vp, vp, vp, vp, vp, vp]
        lib.gks_kinetic_energy.restype = st
        lib.gks_last_error.argtypes = []
        lib.gks_last_error.restype = ctypes.c_char_p
        _lib = lib
    return _lib


def _check(code):
    if code != GKS_OK:
        raise GksError(code, load().gks_last_error().decode(errors="replace"))


def _np(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dp(t):
    return ctypes.c_void_p(t.data_ptr())


def params(precision=FP64, gamma=1.4, cfl=0.5, mu=0.0, Pr=1.0, viscous=False, weno_eps=1e-6, weno_gamma_m=0.0125,
           weno_p=1.0, tau_eps=0.01, tau_C=1.0, force_linear=False, dt_given=False, fallback=False,
           fallback_floor=0.0, smooth=False, mu_power=0.0, T_ref=1.0, bc=None) -> Params:
    """mu_power != 0 (viscous): viscosity mu (T / T_ref)^mu_power at the interface temperature T = p / rho.
    bc: six Boundary records for the box planes x=0, x=L, y=0, y=L, z=0, z=L of a mesh with walls."""
    p = Params()
    load().gks_default_params(ctypes.byref(p))
    p.gamma, p.cfl, p.mu, p.Pr = gamma, cfl, mu, Pr
    p.weno_eps, p.weno_gamma_m, p.weno_p = weno_eps, weno_gamma_m, weno_p
    p.tau_eps, p.tau_C = tau_eps, tau_C
    p.viscous, p.precision, p.force_linear, p.dt_given = int(viscous), int(precision), int(force_linear), int(dt_given)
    p.first_order_fallback = int(fallback)
    p.fallback_floor = float(fallback_floor)
    p.smooth_flux = int(smooth)
    p.mu_power, p.T_ref = float(mu_power), float(T_ref)
    if bc is not None:
        for k in range(6):
            p.bc[k] = bc[k]
    return p


class HostMesh:
    """Host-side preprocessed mesh (connectivity, geometry, stencils, pseudo-inverses, Morton order)."""

    def __init__(self, mesh, min_big: int = 0):
        """min_big > 0 grows big stencils with fewer members like ill-posed fits (0: the paper's set)."""
        lib = load()
        self._nodes = np.ascontiguousarray(mesh.nodes, np.float64)
        self._types = np.ascontiguousarray(mesh.types, np.int8)
        self._cells = np.ascontiguousarray(mesh.cells, np.int64)
        box = np.asarray(mesh.box, np.float64)
        h = ctypes.c_void_p()
        _check(lib.gks_preprocess(self._nodes.shape[0], _np(self._nodes), self._types.shape[0], _np(self._types),
                                  _np(self._cells), _np(box), int(mesh.periodic), int(min_big), ctypes.byref(h)))
        self.h = h
        self._lib = lib  # the library that owns h frees it, also at interpreter shutdown
        n, nf, ns, nsc, ng = (ctypes.c_int64() for _ in range(5))
        _check(lib.gks_host_mesh_counts(h, ctypes.byref(n), ctypes.byref(nf), ctypes.byref(ns), ctypes.byref(nsc),
                                        ctypes.byref(ng)))
        self.n, self.n_faces, self.n_stencil, self.n_grown = n.value, nf.value, ns.value, ng.value
        self.n_subcoef = nsc.value
        self.n_cellfaces = 2 * self.n_faces
        self.perm = np.zeros(self.n, np.int64)
        _check(lib.gks_host_mesh_perm(h, _np(self.perm)))
        self.inv = np.empty_like(self.perm)
        self.inv[self.perm] = np.arange(self.n)

    def geometry(self):
        vol = np.zeros(self.n)
        xc = np.zeros((self.n, 3))
        _check(load().gks_host_mesh_geometry(self.h, _np(vol), _np(xc)))
        return vol, xc

    def faces(self):
        o = np.zeros(self.n_faces, np.int32)
        nb = np.zeros(self.n_faces, np.int32)
        _check(load().gks_host_mesh_faces(self.h, _np(o), _np(nb)))
        return o, nb

    def face_geometry(self):
        """[9, 4 n_faces]: offsets of each Gauss point from the owner's and the neighbour's centroid,
        weighted vector area."""
        g = np.zeros((9, 4 * self.n_faces))
        _check(load().gks_host_mesh_face_geometry(self.h, _np(g)))
        return g

    def to_internal(self, Q):
        """[5, n] in the caller's cell order -> internal order."""
        return np.ascontiguousarray(np.asarray(Q)[:, self.perm])

    def to_external(self, Q):
        out = np.empty_like(Q)
        out[:, self.perm] = Q
        return out

    def __del__(self):
        lib = getattr(self, "_lib", None)
        if lib is not None and getattr(self, "h", None):
            lib.gks_host_mesh_free(self.h)
            self.h = None


class Solver:
    """Device-resident mesh plus work buffer on one GPU; every call enqueues HIP kernels."""

    def __init__(self, host: HostMesh, prm: Params | None = None, device="cuda:0", stream=None):
        import torch

        if not torch.cuda.is_available():
            raise GksError(GKS_EDEVICE, "no GPU available: the gas-kinetic solver runs only on the HIP device")
        lib = load()
        self.torch = torch
        self.host = host
        self.P = prm if prm is not None else params()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        mb, wb, tb = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
        _check(lib.gks_mesh_sizes(host.h, self.P.precision, ctypes.byref(mb), ctypes.byref(wb), ctypes.byref(tb)))
        self.mesh_bytes, self.work_bytes, self.tape_bytes = mb.value, wb.value, tb.value
        self.arena = torch.empty(self.mesh_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.arena.data_ptr()) % 256
        self._arena_ptr = ctypes.c_void_p(self.arena.data_ptr() + off)
        self.work = torch.zeros(self.work_bytes + 256, dtype=torch.uint8, device=self.device)
        self._work_ptr = ctypes.c_void_p(self.work.data_ptr() + ((-self.work.data_ptr()) % 256))
        self.dt = torch.zeros(1, dtype=torch.float64, device=self.device)
        m = ctypes.c_void_p()
        _check(lib.gks_init_mesh(host.h, self.P.precision, self._arena_ptr, self.mesh_bytes, self._s(),
                                 ctypes.byref(m)))
        self.m = m
        self._lib = lib  # the library that owns m destroys it, also at interpreter shutdown
        self.n, self.n_faces = host.n, host.n_faces
        cdt = torch.float64 if self.P.precision == FP64 else torch.float32
        self.coeff_dtype = cdt
        _check(lib.gks_reset_status(self.m, self._work_ptr, self._s()))

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def __del__(self):
        lib = getattr(self, "_lib", None)
        if lib is not None and getattr(self, "m", None):
            lib.gks_destroy_mesh(self.m)
            self.m = None

    # tensors ---------------------------------------------------------------
    def upload(self, Q_internal: np.ndarray):
        return self.torch.tensor(np.ascontiguousarray(Q_internal, np.float64), device=self.device)

    def _q(self, Q):
        assert Q.dtype == self.torch.float64 and Q.is_contiguous() and Q.shape == (5, self.n)
        return _dp(Q)

    # entry points ----------------------------------------------------------
    def timestep(self, Q):
        _check(load().gks_timestep(self.m, self._q(Q), ctypes.byref(self.P), _dp(self.dt), self._work_ptr, self._s()))
        return self.dt

    def reconstruct(self, Q):
        coeff = self.torch.empty((self.n, 5, 10), dtype=self.coeff_dtype, device=self.device)
        _check(load().gks_reconstruct(self.m, self._q(Q), _dp(coeff), ctypes.byref(self.P), self._work_ptr,
                                      self._s()))
        return coeff

    def flux(self, coeff, Q, dt):
        if not isinstance(dt, self.torch.Tensor):
            self.dt.fill_(float(dt))
            dt = self.dt
        ff = self.torch.empty((self.n_faces, 10), dtype=self.coeff_dtype, device=self.device)
        _check(load().gks_flux(self.m, _dp(coeff), self._q(Q), _dp(dt), _dp(ff), ctypes.byref(self.P),
                               self._work_ptr, self._s()))
        return ff

    def residual(self, ff):
        L = self.torch.empty((5, self.n), dtype=self.torch.float64, device=self.device)
        D = self.torch.empty_like(L)
        _check(load().gks_residual(self.m, _dp(ff), _dp(L), _dp(D), ctypes.byref(self.P), self._s()))
        return L, D

    def coeff_tape(self):
        """A device buffer for both stages' reconstructions of one step (tape_bytes_per_step)."""
        return self.torch.empty(self.tape_bytes // self.coeff_dtype.itemsize, dtype=self.coeff_dtype,
                                device=self.device)

    def step(self, Q, dt=None, Q_star=None, coeff_tape=None):
        """One S2O4 step in place; dt=None computes the CFL step on the device."""
        if dt is None:
            self.P.dt_given = 0
        else:
            self.dt.fill_(float(dt))
            self.P.dt_given = 1
        qs = _dp(Q_star) if Q_star is not None else None
        tape = _dp(coeff_tape) if coeff_tape is not None else None
        _check(load().gks_s2o4_step(self.m, self._q(Q), _dp(self.dt), ctypes.byref(self.P), self._work_ptr, qs,
                                    tape, self._s()))
        self.P.dt_given = 0
        return Q

    def step_noalloc(self, Q, status, dt=None, Q_star=None, coeff_tape=None):
        """One S2O4 step in place through the allocation-free entry point: the library's static scratch
        replaces the work buffer; status is a caller-owned int32[2] device tensor (sticky non-physical
        flag, fallback count) that the call never clears."""
        assert status.dtype == self.torch.int32 and status.numel() >= 2 and status.device == self.device
        if dt is None:
            self.P.dt_given = 0
        else:
            self.dt.fill_(float(dt))
            self.P.dt_given = 1
        qs = _dp(Q_star) if Q_star is not None else None
        tape = _dp(coeff_tape) if coeff_tape is not None else None
        try:
            _check(load().gks_s2o4_step_noalloc(self.m, self._q(Q), _dp(self.dt), ctypes.byref(self.P), _dp(status),
                                                qs, tape, self._s()))
        finally:
            self.P.dt_given = 0
        return Q

    def implicit_step(self, Q, dt_factor=10.0, kmax=3, dt=None):
        """One implicit Jacobi step in place: the GKS residual over the flux step (the CFL step, or dt),
        the implicit operator with the pseudo-time step dt_factor times it, kmax sweeps."""
        if dt is None:
            self.P.dt_given = 0
        else:
            self.dt.fill_(float(dt))
            self.P.dt_given = 1
        _check(load().gks_implicit_step(self.m, self._q(Q), _dp(self.dt), float(dt_factor), int(kmax),
                                        ctypes.byref(self.P), self._work_ptr, self._s()))
        self.P.dt_given = 0
        return Q

    # adjoint -------------------------------------------------------------
    def _adj_work(self):
        if getattr(self, "adj_work", None) is None:
            b = ctypes.c_size_t()
            _check(load().gks_adjoint_work_bytes(self.host.h, ctypes.byref(b)))
            self.adj_work = self.torch.empty(b.value + 256, dtype=self.torch.uint8, device=self.device)
            self._adj_ptr = ctypes.c_void_p(self.adj_work.data_ptr() + ((-self.adj_work.data_ptr()) % 256))
        return self._adj_ptr

    def adjoint_step(self, Qn, Qstar, dt, lam_next, lam_out=None, coeff_tape=None):
        """lam_n from lam_{n+1} for the S2O4 step Qn -> (Qstar) -> Q_{n+1}; dt: 1-element device tensor;
        coeff_tape: that step's tape from step/step_to (optional: the reconstructions are recomputed)."""
        lam_out = self.torch.empty_like(lam_next) if lam_out is None else lam_out
        tape = _dp(coeff_tape) if coeff_tape is not None else None
        _check(load().gks_adjoint_step(self.m, self._q(Qn), self._q(Qstar), _dp(dt), self._q(lam_next),
                                       self._q(lam_out), ctypes.byref(self.P), self._adj_work(), tape, self._s()))
        return lam_out

    def kinetic_energy(self, Q, grad=False):
        """(J, dJ/dQ or None): J = sum |Omega| |rho U|^2 / (2 rho), on the device."""
        J = self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        g = self.torch.empty_like(Q) if grad else None
        _check(load().gks_kinetic_energy(self.m, self._q(Q), _dp(J), _dp(g) if grad else None, self._work_ptr,
                                         self._s()))
        return J, g

    def step_to(self, Q, dt_ptr_tensor, Q_star=None, coeff_tape=None):
        """One S2O4 step in place with dt read from a 1-element device tensor (no host round trip)."""
        self.P.dt_given = 1
        qs = _dp(Q_star) if Q_star is not None else None
        tape = _dp(coeff_tape) if coeff_tape is not None else None
        try:
            _check(load().gks_s2o4_step(self.m, self._q(Q), _dp(dt_ptr_tensor), ctypes.byref(self.P),
                                        self._work_ptr, qs, tape, self._s()))
        finally:
            self.P.dt_given = 0
        return Q

    def set_flux_window(self, cells: int):
        """Testing aid: narrow the owner window of the FP64 periodic flux kernel to `cells` in [0, 92]
        (owners beyond it are read from memory directly; results are bitwise the same)."""
        _check(load().gks_set_flux_window(self.m, int(cells)))

    def profile(self, enable=True):
        """Record HIP events around every kernel launch of this solver (host-side events)."""
        _check(load().gks_profile(self.m, int(enable)))

    def profile_read(self):
        """{kernel: (total ms, launches)} since the last read; synchronises."""
        ms = np.zeros(len(KERNELS))
        cnt = np.zeros(len(KERNELS), np.int64)
        _check(load().gks_profile_read(self.m, _np(ms), _np(cnt)))
        return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KERNELS)}

    def poll(self):
        _check(load().gks_poll_status(self.m, self._work_ptr, self._s()))

    def fallback_count(self):
        """Gauss-point side states that fell back to first order since the last call (synchronises)."""
        c = ctypes.c_int64()
        _check(load().gks_fallback_count(self.m, self._work_ptr, ctypes.byref(c), self._s()))
        return c.value

    def run(self, Q, nsteps=0, t_end=0.0):
        """Advance nsteps steps, or to t_end with the last step shortened; returns the step sizes."""
        dts = []
        t = 0.0
        while True:
            if t_end > 0:
                if t >= t_end * (1 - 1e-14):
                    break
            elif len(dts) >= nsteps:
                break
            if t_end > 0:
                # the time step kernel caps the CFL step at the time left, so the last step lands on t_end
                self.P.dt_max = t_end - t
                try:
                    self.step(Q)
                finally:
                    self.P.dt_max = 0.0
                # the step size is read back for the clock: stop at the first non-physical state instead
                # of marching a broken field with ever smaller steps
                dt = float(self.dt.item())
                self.poll()
                if not (math.isfinite(dt) and dt > 0.0):
                    raise GksError(GKS_ENONPHYS, f"time step {dt} at t = {t}")
            else:
                self.step(Q)
                dt = None
            dts.append(dt)
            if dt is not None:
                t += dt
        if t_end > 0:
            self.poll()
        return dts


def gp_op_count(viscous=False, Pr=1.0):
    """Operations of one Gauss point of the flux kernel: dict(add, mul, div, transc)."""
    v = [ctypes.c_int64() for _ in range(4)]
    _check(load().gks_gp_op_count(int(viscous), Pr, *(ctypes.byref(x) for x in v)))
    return dict(add=v[0].value, mul=v[1].value, div=v[2].value, transc=v[3].value)


def gp_flux_batch(ql, dql, qr, dqr, dt, precision=FP64, **kw):
    """Single Gauss-point fluxes on the GPU for a batch of local-frame states (numpy in, numpy out)."""
    import torch

    n = ql.shape[0]
    dev = torch.device("cuda:0")
    t = [torch.tensor(np.ascontiguousarray(a, np.float64), device=dev) for a in (ql, dql, qr, dqr, dt)]
    out = torch.zeros((n, 10), dtype=torch.float64, device=dev)
    prm = params(precision=precision, **kw)
    _check(load().gks_gp_flux_batch(n, *(_dp(a) for a in t), _dp(out), ctypes.byref(prm),
                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)))
    torch.cuda.synchronize()
    return out.cpu().numpy()
