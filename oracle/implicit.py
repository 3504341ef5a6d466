"""Implicit Jacobi step of the steady solver (Section 3.3: Eq. impEuler, Eq. euler-scheme, Eq. jacobi).

Test infrastructure: a plain numpy statement of the step on top of the oracle's own
residual (reconstruction + GKS flux, Eq. finite); the GPU library never imports it.

One step from Q^n with pseudo-time step dt:
- Res_i = the GKS flux balance averaged over a time step dt_f:
  Res = -(1 / (dt_f |Omega_i|)) sum_f int_0^dt_f F_f dt = L + dt_f/2 dL/dt.  The paper writes one
  dt for both; the time evolution of the GKS flux is only meaningful over a step of the explicit
  scheme's size, and with dt_f = dt at 10-20 times that step the flux's time derivative,
  extrapolated over dt, makes the iteration leave the physical states (a viscous decay problem on
  the hybrid lattice, measured here).  So dt_f is the explicit CFL step and dt = (a factor) x dt_f
  enters only the implicit operator; with the factor 1 this is the printed form;
- the implicit operator is the flux-split one of Eq. euler-scheme: across face f of cell i,
  with outward normal n and area S, 1/2 (T(Q_nb) + T(Q_i) - r (Q_nb - Q_i)) S, where T(Q) is
  the Euler flux of Q along n and r = |U_nb . n| + c_nb (the neighbour's state at t_n);
- the paper prints the flux-split operator without the 1/|Omega_i| that Res carries; both
  sides are taken per unit volume consistently, i.e. multiplied by |Omega_i|:
      D_i dQ_i + 1/2 sum_f [T(Q_nb + dQ_nb) - T(Q_nb) - r dQ_nb] S = |Omega_i| Res_i,
      D_i = |Omega_i| / dt + 1/2 sum_f r S
  (the cell's own T(Q_i) terms cancel: T is linear in n and a closed cell's areas sum to 0);
- Jacobi: dQ^(0) = |Omega| Res / D, then k_max sweeps with the neighbours' previous iterate;
  Q^{n+1} = Q^n + dQ^(k_max);
- a face on a box plane of a mesh with walls has as neighbour the ghost of Section 2's
  construction: the plane's condition applied to the cell's own state, Q_nb = B(Q_i); its
  increment is that of the condition applied to the cell's updated state,
  dQ_nb = B(Q_i + dQ_i) - B(Q_i), with the cell's previous iterate in each sweep (the paper's
  implicit cases have walls but print no ghost treatment for the implicit operator).
"""
from __future__ import annotations

import numpy as np

import oracle


def euler_flux(Q: np.ndarray, n: np.ndarray, gamma: float) -> np.ndarray:
    """Euler flux of the states Q [5, m] along the unit normals n [m, 3]."""
    rho, mom, E = Q[0], Q[1:4], Q[4]
    U = mom / rho
    un = (U * n.T).sum(axis=0)
    p = (gamma - 1.0) * (E - 0.5 * (mom * U).sum(axis=0))
    T = np.empty_like(Q)
    T[0] = rho * un
    T[1:4] = mom * un + p * n.T
    T[4] = (E + p) * un
    return T


def face_normals(o):
    """Per face: unit normal (owner -> neighbour) and area, from the Gauss points' weighted vector areas."""
    fi = o.face_info()
    va = fi["va"]
    A = va.sum(axis=1)
    S = np.linalg.norm(va, axis=2).sum(axis=1)
    return fi["owner"], fi["nbr"], A / np.linalg.norm(A, axis=1)[:, None], S


def wall_planes(nf: np.ndarray) -> np.ndarray:
    """Box plane (2 axis + hi) of wall faces with outward unit normals nf [m, 3]: the axis the normal
    lies along, hi where it points up that axis (the plane x_axis = L)."""
    d = np.abs(nf).argmax(axis=1)
    return 2 * d + (nf[np.arange(len(d)), d] > 0)


def ghosts(prm, planes: np.ndarray, V: np.ndarray) -> np.ndarray:
    """The condition of each face's plane on the matching column of the cell averages V [5, m]."""
    out = np.empty_like(V)
    for j, pl in enumerate(planes):
        out[:, j] = oracle.bc_ghost(prm, int(pl), V[:, j], np.zeros((5, 3)))[0]
    return out


def jacobi_step(o, Q: np.ndarray, dt: float, kmax: int = 3, gamma: float = 1.4, dt_flux: float | None = None) -> np.ndarray:
    """Q^{n+1} of one implicit step of pseudo-time step dt on the oracle `o` (whose parameters set the
    GKS flux and the box planes' conditions); the flux is integrated over dt_flux (default dt)."""
    dt_flux = dt if dt_flux is None else dt_flux
    n = Q.shape[1]
    owner, nbr, nf, S = face_normals(o)
    wall = nbr < 0
    L, D = o.residual(Q, dt_flux)
    res = L + 0.5 * dt_flux * D
    vol = o.cell_geometry()[0]
    # every interior face seen from each of its two cells and every wall face from its cell:
    # (cell, neighbour, outward normal, area); a wall face's neighbour is the ghost of its cell
    inner = ~wall
    cell = np.r_[owner[inner], nbr[inner], owner[wall]]
    other = np.r_[nbr[inner], owner[inner], owner[wall]]
    nout = np.r_[nf[inner], -nf[inner], nf[wall]]
    S2 = np.r_[S[inner], S[inner], S[wall]]
    ng = int(wall.sum())
    planes = wall_planes(nf[wall])
    gslot = slice(len(cell) - ng, len(cell))

    Qo = Q[:, other]
    if ng:
        Qo[:, gslot] = ghosts(o.P, planes, Qo[:, gslot])
    rho = Qo[0]
    U = Qo[1:4] / rho
    p = (gamma - 1.0) * (Qo[4] - 0.5 * rho * (U * U).sum(axis=0))
    r = np.abs((U * nout.T).sum(axis=0)) + np.sqrt(gamma * p / rho)
    diag = vol / dt + 0.5 * np.bincount(cell, weights=r * S2, minlength=n)
    T0 = euler_flux(Qo, nout, gamma)
    b = vol * res
    dQ = b / diag
    for _ in range(kmax):
        dQo = dQ[:, other]
        Q1 = Qo + dQo
        if ng:  # a ghost's increment: the condition on the cell's updated state
            Q1[:, gslot] = ghosts(o.P, planes, Q[:, other[gslot]] + dQo[:, gslot])
            dQo[:, gslot] = Q1[:, gslot] - Qo[:, gslot]
        term = (euler_flux(Q1, nout, gamma) - T0 - r * dQo) * S2
        off = np.stack([np.bincount(cell, weights=term[c], minlength=n) for c in range(5)])
        dQ = (b - 0.5 * off) / diag
    return Q + dQ


def residual_norm(o, Q: np.ndarray, dt: float) -> float:
    """Volume-weighted L1 norm of the density residual (the steady solver's convergence measure)."""
    L, D = o.residual(Q, dt)
    vol = o.cell_geometry()[0]
    return float((np.abs(L[0] + 0.5 * dt * D[0]) * vol).sum())
