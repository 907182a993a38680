"""Differentiable IMEX rollouts: a torch.autograd.Function over the library's
forward step and its hand-written adjoint (``imexlb_adjoint_step``).

The forward pass starts from the local equilibrium of the initial fields
(n, u_x, u_y, T), runs nsteps IMEX steps in the library and keeps a copy of
the state every ``every`` steps.  The backward pass seeds the adjoint from
the gradients of the final moments (``imexlb_moments_adjoint``), then walks
the segments backwards: each segment is recomputed forward from its
checkpoint, storing its states and each step's stage sources and moments
(``imexlb_step_recorded``), and the adjoint steps run through them in
reverse without recomputing those (``imexlb_adjoint_step_recorded``); the
equilibrium adjoint (``imexlb_equilibrium_adjoint``) finally
maps the adjoint state to gradients of the initial fields.  The density loss
and its gradient come from ``imexlb_density_loss``.  Every step of this runs
in the library's HIP kernels; this module only orders the calls and holds
the checkpoints.
"""
from __future__ import annotations

import torch

from . import imexlb as I


def _zeros_like_field(solver):
    return torch.zeros(solver.cfg.field_shape, dtype=torch.float64, device=solver.device)


class EquilibriumRollout(torch.autograd.Function):
    """(n0, ux0, uy0, T0) -> (n, ux, uy, T) after nsteps steps from the
    equilibrium of the initial fields (FP64 device tensors of the grid's
    field shape; uy is ignored and returned as zeros when d = 1)."""

    @staticmethod
    def forward(ctx, n0, ux0, uy0, T0, solver, nsteps: int, every: int):
        every = max(1, int(every))
        solver.set_equilibrium(n0.detach(), ux0.detach(), uy0.detach(), T0.detach())
        checkpoints = []
        for k in range(nsteps):
            if k % every == 0:
                checkpoints.append(solver.state.clone())
            solver.step(1)
        final_state = solver.state.clone()
        n, ux, uy, T = solver.moments()
        ctx.solver, ctx.nsteps, ctx.every = solver, nsteps, every
        ctx.checkpoints, ctx.final_state = checkpoints, final_state
        ctx.save_for_backward(n0.detach(), ux0.detach(), uy0.detach(), T0.detach())
        return n, ux, uy, T

    @staticmethod
    def backward(ctx, gn, gux, guy, gT):
        s = ctx.solver
        n0, ux0, uy0, T0 = ctx.saved_tensors
        g = [x if x is not None else _zeros_like_field(s) for x in (gn, gux, guy, gT)]
        lam = s.moments_adjoint(ctx.final_state, *g)
        nseg = len(ctx.checkpoints)
        for seg in reversed(range(nseg)):
            start = seg * ctx.every
            end = min(start + ctx.every, ctx.nsteps)
            s.set_state(ctx.checkpoints[seg])
            states, records = [], []
            for _ in range(start, end):
                states.append(s.state.clone())
                records.append(s.new_record())
                s.step_recorded(records[-1])
            for F, rec in zip(reversed(states), reversed(records)):
                lam = s.adjoint_step(F, lam, record=rec)
        dn, dux, duy, dT = s.equilibrium_adjoint(n0, ux0, uy0, T0, lam)
        return dn, dux, duy, dT, None, None, None


class DensityLoss(torch.autograd.Function):
    """n -> 1/2 sum (n - target)^2 in the library (``imexlb_density_loss``),
    with dL/dn = n - target from the same call."""

    @staticmethod
    def forward(ctx, n, target, solver):
        loss, grad = solver.density_loss(target.detach(), n=n.detach(), grad=True)
        ctx.save_for_backward(grad)
        return loss

    @staticmethod
    def backward(ctx, gloss):
        (grad,) = ctx.saved_tensors
        return gloss * grad, None, None


def rollout(solver, n0, ux0, uy0, T0, nsteps: int, every: int = 20):
    """Differentiable final moments of an nsteps rollout (see
    EquilibriumRollout)."""
    if uy0 is None:
        uy0 = torch.zeros_like(n0)
    return EquilibriumRollout.apply(n0, ux0, uy0, T0, solver, nsteps, every)


def density_loss_gradient(solver, n0, target, nsteps: int, every: int = 20, P: float = 1.0):
    """Loss 1/2 sum (n - target)^2 after nsteps from n = n0, u = 0, P fixed
    (T = P / n0), and its gradient with respect to n0."""
    n0 = n0.detach().clone().requires_grad_(True)
    zero = torch.zeros_like(n0)
    T0 = P / n0
    n, _, _, _ = rollout(solver, n0, zero, zero, T0, nsteps, every)
    loss = DensityLoss.apply(n, target, solver)
    loss.backward()
    return float(loss.detach()), n0.grad.detach()


__all__ = ["EquilibriumRollout", "DensityLoss", "rollout", "density_loss_gradient", "I"]
