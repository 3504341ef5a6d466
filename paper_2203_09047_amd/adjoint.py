"""Checkpointed discrete adjoint of an S2O4 rollout behind torch.autograd.

``Rollout.apply(Q0, solver, nsteps, ckpt_every)`` advances Q0 by nsteps CFL
steps on the GPU and returns the final state; its backward propagates the
cotangent of the final state to Q0 with the library's hand-written adjoint
(``gks_adjoint_step``), recomputing each segment of ``ckpt_every`` steps from
its checkpoint.  The step sizes chosen in the forward pass are frozen.  The
recomputation keeps each step's reconstructions (a coefficient tape of
800 bytes per cell per step in FP64) so the adjoint does not redo them; with
``keep_coefficients=False`` the adjoint recomputes them instead.

``store_all=True`` trades memory for the recomputation: the forward pass keeps
every step's start state, stage state and coefficient tape (880 bytes per cell
per step in FP64: 16 GB for 100 steps of 180 k cells, 26 GB for 20 steps of
1.47 M cells, well inside one GPU's HBM), and the backward runs the adjoint
steps only.
"""
from __future__ import annotations

import torch


class Rollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, Q0, solver, nsteps, ckpt_every=10, keep_coefficients=True, store_all=False):
        Q = Q0.detach().clone()
        dts = torch.zeros(max(nsteps, 1), dtype=torch.float64, device=Q.device)
        ckpts, states = {}, []
        for k in range(nsteps):
            if store_all:
                Qn, Qs, tape = Q.clone(), torch.empty_like(Q), solver.coeff_tape()
                solver.step(Q, Q_star=Qs, coeff_tape=tape)
                states.append((Qn, Qs, tape))
            else:
                if k % ckpt_every == 0:
                    ckpts[k] = Q.clone()
                solver.step(Q)                   # CFL dt computed on the device into solver.dt
            dts[k:k + 1].copy_(solver.dt)        # frozen for the adjoint
        ctx.solver, ctx.nsteps, ctx.ckpt_every = solver, nsteps, ckpt_every
        ctx.keep = keep_coefficients
        ctx.ckpts, ctx.dts, ctx.states = ckpts, dts, states
        return Q

    @staticmethod
    def backward(ctx, grad_out):
        solver, nsteps, every = ctx.solver, ctx.nsteps, ctx.ckpt_every
        lam = grad_out.detach().contiguous().clone()
        lam_tmp = torch.empty_like(lam)
        if ctx.states:  # every step kept by the forward pass: no recomputation
            for k in reversed(range(nsteps)):
                Qn, Qs, tape = ctx.states[k]
                solver.adjoint_step(Qn, Qs, ctx.dts[k:k + 1], lam, lam_tmp, coeff_tape=tape)
                lam, lam_tmp = lam_tmp, lam
                ctx.states[k] = None
            return lam, None, None, None, None, None
        for seg in reversed(range(0, nsteps, every)):
            last = min(seg + every, nsteps)
            # recompute the segment, keeping each step's start state and stage state
            Q = ctx.ckpts[seg].clone()
            states = []
            for k in range(seg, last):
                Qn = Q.clone()
                Qs = torch.empty_like(Q)
                tape = solver.coeff_tape() if ctx.keep else None
                solver.step_to(Q, ctx.dts[k:k + 1], Q_star=Qs, coeff_tape=tape)
                states.append((Qn, Qs, tape))
            for k in reversed(range(seg, last)):
                Qn, Qs, tape = states[k - seg]
                solver.adjoint_step(Qn, Qs, ctx.dts[k:k + 1], lam, lam_tmp, coeff_tape=tape)
                lam, lam_tmp = lam_tmp, lam
                states[k - seg] = None
        return lam, None, None, None, None, None


def kinetic_energy_gradient(solver, Q0, nsteps, ckpt_every=10, store_all=False):
    """(J, dJ/dQ0) of the kinetic energy after nsteps steps from Q0."""
    Q0 = Q0.detach().clone().requires_grad_(True)
    QT = Rollout.apply(Q0, solver, nsteps, ckpt_every, True, store_all)
    J, g = solver.kinetic_energy(QT.detach(), grad=True)
    QT.backward(g)
    return J, Q0.grad
