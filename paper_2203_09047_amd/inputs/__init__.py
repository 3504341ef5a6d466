"""Seeded synthetic inputs: hybrid-lattice meshes and cell-averaged fields.

This module holds none of the numerical method's arithmetic.  It is the one
source of inputs shared by the GPU library's tests and benchmark and by the
FP64 reference, so that both see identical meshes and initial data.

Mesh records follow the paper's cell labels (Section 2): ``types`` uses
0 = tetrahedron, 1 = pyramid, 2 = prism, 3 = hexahedron and ``cells`` holds
up to 8 node ids per cell (-1 padded) in the paper's vertex order.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgks_inputs.so")
SOURCE = os.path.join(_HERE, "gks_inputs.c")

KINDS = {"hybrid": 0, "hex": 1, "tet": 2, "pyr": 3, "prism": 4, "hexprism": 5}
TYPE_NAMES = ("tet", "pyr", "prism", "hex")
MESH_SEED = 2203
PERTURB_SEED = 9047

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the C generator with gcc (host only)."""
    import subprocess

    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-o", LIB_PATH, SOURCE, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        lib = ctypes.CDLL(LIB_PATH)
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.c_void_p
        lib.gin_lattice.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, dp, i64p, i64p, dp, dp,
                                    dp, dp]
        lib.gin_lattice.restype = ctypes.c_int
        lib.gin_cell_averages.argtypes = [ctypes.c_int64, dp, dp, dp, ctypes.c_int, ctypes.c_double, dp, ctypes.c_int,
                                          dp, ctypes.c_int, dp]
        lib.gin_cell_averages.restype = ctypes.c_int
        lib.gin_splitmix64.argtypes = [ctypes.c_uint64]
        lib.gin_splitmix64.restype = ctypes.c_uint64
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Mesh:
    nodes: np.ndarray        # [n_nodes, 3] float64
    types: np.ndarray        # [n_cells] int8
    cells: np.ndarray        # [n_cells, 8] int64, -1 padded
    box: tuple               # (Lx, Ly, Lz)
    periodic: bool
    N: int = 0
    kind: str = "hybrid"
    seed: int = MESH_SEED
    hist: dict = field(default_factory=dict)

    @property
    def n_cells(self) -> int:
        return int(self.types.shape[0])


def lattice(N: int, kind: str = "hybrid", seed: int = MESH_SEED, box=(1.0, 1.0, 1.0), periodic: bool = True) -> Mesh:
    """Build the N^3 lattice mesh of the given kind on [0,Lx]x[0,Ly]x[0,Lz]."""
    lib = _load()
    boxa = np.asarray(box, dtype=np.float64)
    nn = ctypes.c_int64()
    nc = ctypes.c_int64()
    hist = np.zeros(4, np.int64)
    rc = lib.gin_lattice(N, KINDS[kind], seed, int(periodic), _ptr(boxa), ctypes.byref(nn), ctypes.byref(nc),
                         _ptr(hist), None, None, None)
    if rc:
        raise ValueError("bad lattice arguments")
    nodes = np.zeros((nn.value, 3), np.float64)
    types = np.zeros(nc.value, np.int8)
    cells = np.full((nc.value, 8), -1, np.int64)
    rc = lib.gin_lattice(N, KINDS[kind], seed, int(periodic), _ptr(boxa), ctypes.byref(nn), ctypes.byref(nc),
                         _ptr(hist), _ptr(nodes), _ptr(types), _ptr(cells))
    if rc:
        raise ValueError("bad lattice arguments")
    h = {TYPE_NAMES[t]: int(hist[t]) for t in range(4)}
    return Mesh(nodes, types, cells, tuple(float(b) for b in box), bool(periodic), N, kind, seed, h)


# ----------------------------------------------------------------------------
# fields
# ----------------------------------------------------------------------------
@dataclass
class Field:
    kind: int
    params: np.ndarray
    modes: np.ndarray | None = None


def wave(amp=0.2, k=(2 * math.pi, 2 * math.pi, 2 * math.pi), U=(1.0, 1.0, 1.0), p0=1.0, t=0.0) -> Field:
    """rho = 1 + amp sin(k.(x - U t)), velocity U, pressure p0."""
    p = np.zeros(16)
    p[0] = amp
    p[1:4] = k
    p[4:7] = U
    p[7] = p0
    p[8] = t
    return Field(0, p)


def tgv(V0=1.0, rho0=1.0, mach=0.1, gamma=1.4) -> Field:
    """Taylor-Green vortex on [0, 2 pi]^3 with p0 = rho0 V0^2 / (gamma Ma^2)."""
    p = np.zeros(16)
    p[0] = V0
    p[1] = rho0
    p[2] = rho0 * V0 * V0 / (gamma * mach * mach)
    return Field(1, p)


def riemann(normal=(1.0, 0.3, 0.2), c=0.6, left=(1.0, 0, 0, 0, 1.0), right=(0.125, 0, 0, 0, 0.1)) -> Field:
    """Two primitive states (rho,u,v,w,p) split by the plane normal.x = c."""
    p = np.zeros(16)
    p[0:3] = normal
    p[3] = c
    p[4:9] = left
    p[9:14] = right
    return Field(2, p)


def uniform(rho=1.0, u=0.0, v=0.0, w=0.0, p=1.0) -> Field:
    q = np.zeros(16)
    q[0:5] = (rho, u, v, w, p)
    return Field(4, q)


def gaussian(seed: int, n: int) -> np.ndarray:
    """n standard normal draws from SplitMix64 (Box-Muller)."""
    lib = _load()
    out = np.empty(n)
    state = seed
    i = 0
    while i < n:
        state = lib.gin_splitmix64(state)
        u1 = ((state >> 11) + 0.5) / float(1 << 53)
        state = lib.gin_splitmix64(state)
        u2 = ((state >> 11) + 0.5) / float(1 << 53)
        r = math.sqrt(-2.0 * math.log(u1))
        out[i] = r * math.cos(2 * math.pi * u2)
        if i + 1 < n:
            out[i + 1] = r * math.sin(2 * math.pi * u2)
        i += 2
    return out


def perturbed_wave(amp=0.2, U=(1.0, 1.0, 1.0), p0=1.0, kmax=4, rms=0.05, seed=PERTURB_SEED) -> Field:
    """Density wave plus a seeded low-pass velocity perturbation.

    u' = sum_n A_n cos(2 pi n.x) + B_n sin(2 pi n.x) over integer n in a half
    space with 0 < |n| <= kmax, A_n, B_n in R^3 iid N(0,1), scaled so each
    velocity component has the given RMS over the unit cube.
    """
    ns = []
    for a in range(-kmax, kmax + 1):
        for b in range(-kmax, kmax + 1):
            for c in range(-kmax, kmax + 1):
                n2 = a * a + b * b + c * c
                if n2 == 0 or n2 > kmax * kmax:
                    continue
                if (a, b, c) <= (0, 0, 0) and (a < 0 or (a == 0 and (b < 0 or (b == 0 and c < 0)))):
                    continue
                ns.append((a, b, c))
    g = gaussian(seed, 6 * len(ns)).reshape(len(ns), 6)
    # RMS of component q over the cube: sqrt(sum_n (A_nq^2 + B_nq^2) / 2)
    rms_now = np.sqrt(0.5 * (g[:, 0:3] ** 2 + g[:, 3:6] ** 2).sum(axis=0))
    g[:, 0:3] *= rms / rms_now
    g[:, 3:6] *= rms / rms_now
    modes = np.zeros((len(ns), 9))
    modes[:, 0:3] = np.asarray(ns, float)
    modes[:, 3:9] = g
    f = wave(amp, (2 * math.pi,) * 3, U, p0)
    f.kind = 3
    f.modes = modes
    return f


def cell_averages(mesh: Mesh, fld: Field, gamma: float = 1.4, order: int = 5) -> np.ndarray:
    """Cell averages [5, n_cells] of (rho, rho U, rho V, rho W, rho E)."""
    lib = _load()
    out = np.zeros((5, mesh.n_cells), np.float64)
    modes = fld.modes if fld.modes is not None else np.zeros((0, 9))
    modes = np.ascontiguousarray(modes, np.float64)
    rc = lib.gin_cell_averages(mesh.n_cells, _ptr(mesh.nodes), _ptr(mesh.types), _ptr(mesh.cells), fld.kind, gamma,
                               _ptr(fld.params), int(modes.shape[0]), _ptr(modes), order, _ptr(out))
    if rc:
        raise ValueError("bad quadrature order")
    return out
