"""Differentiable IMEX rollouts: a torch.autograd.Function over the library's
forward step and its hand-written adjoint (``imexlb_adjoint_step``).

The forward pass starts from the local equilibrium of the initial fields
(n, u_x, u_y, T), runs nsteps IMEX steps in the library and keeps a copy of
the state every ``every`` steps.  The last segment is taken with recorded
out-of-place steps (``imexlb_step_recorded_to``): its states and each step's
stage sources and moments stay on the device, so the reverse sweep starts
without a recomputation.  The backward pass seeds the adjoint from the
gradients of the final moments (``imexlb_moments_adjoint``), then walks the
segments backwards: each earlier segment is recomputed forward from its
checkpoint with recorded out-of-place steps, and the adjoint steps run
through the records in reverse (``imexlb_adjoint_step_recorded``).  The
recomputation of segment k - 1 runs on a second stream while the adjoint
runs through segment k on the caller's stream (they touch disjoint
buffers: the recomputation the solver's workspace, its own records and
states; the adjoint those of segment k and the adjoint workspace).  Both the
recorded last segment and the look-ahead hold whole segments of records on
the device (a record holds five plane-sets and three moment sets), so each is
used only when it fits a memory budget: ``solver.rollout_memory`` bytes when
that attribute is set, else 80 % of the device memory free when the pass
starts; without room the segments are recomputed one at a time on the
caller's stream (the same gradients; to rounding when the last segment, too,
is recomputed, since its first step then starts from the moment kernel's
moments rather than from those of the previous step's last pass).  The
equilibrium adjoint (``imexlb_equilibrium_adjoint``) finally maps the
adjoint state to gradients of the initial fields.  The density loss and its
gradient come from ``imexlb_density_loss``.  Every step of this runs in the
library's HIP kernels; this module only orders the calls and holds the
checkpoints.
"""
from __future__ import annotations

import torch

from . import imexlb as I


def _zeros_like_field(solver):
    return torch.zeros(solver.cfg.field_shape, dtype=torch.float64, device=solver.device)


def _segment_bytes(solver, nsteps: int) -> int:
    """Device bytes of a recorded segment of nsteps steps: its records and
    the states before each step."""
    L, h = solver.L, solver._h
    return nsteps * (L.imexlb_step_record_bytes(h) + L.imexlb_state_bytes(h))


def _memory_budget(solver) -> int:
    """Bytes the rollout may hold in recorded segments: ``solver.rollout_memory``
    when set, else 80 % of the device memory free now (the caching allocator's
    free blocks included)."""
    budget = getattr(solver, "rollout_memory", None)
    if budget is not None:
        return int(budget)
    free, _ = torch.cuda.mem_get_info(solver.device)
    reserved = torch.cuda.memory_reserved(solver.device) - torch.cuda.memory_allocated(solver.device)
    return int(0.8 * (free + reserved))


def _recorded_segment(solver, nsteps: int):
    """nsteps recorded out-of-place steps from the bound state on the
    solver's stream: the states F^k before each step (the first is the
    tensor bound on entry) and the records of the steps."""
    states, records = [], []
    for _ in range(nsteps):
        states.append(solver.state)
        records.append(solver.new_record())
        solver.step_recorded(records[-1], out=torch.empty_like(solver.state))
    return states, records


class EquilibriumRollout(torch.autograd.Function):
    """(n0, ux0, uy0, T0) -> (n, ux, uy, T) after nsteps steps from the
    equilibrium of the initial fields (FP64 device tensors of the grid's
    field shape; uy is ignored and returned as zeros when d = 1)."""

    @staticmethod
    def forward(ctx, n0, ux0, uy0, T0, solver, nsteps: int, every: int):
        every = max(1, int(every))
        need = any(ctx.needs_input_grad[:4])
        solver.set_equilibrium(n0.detach(), ux0.detach(), uy0.detach(), T0.detach())
        checkpoints, tail = [], None
        if not need:
            solver.step(nsteps)
        else:
            nseg = (nsteps + every - 1) // every
            tail0 = (nseg - 1) * every if nseg else nsteps
            # the last segment is recorded here only when it fits the budget;
            # otherwise it gets a checkpoint and is recomputed like the others
            if tail0 < nsteps and _segment_bytes(solver, nsteps - tail0) > _memory_budget(solver):
                tail0 = nsteps
            for k in range(tail0):
                if k % every == 0:
                    checkpoints.append(solver.state.clone())
                solver.step(1)
            if tail0 < nsteps:
                tail = _recorded_segment(solver, nsteps - tail0)
        final_state = solver.state.clone()
        n, ux, uy, T = solver.moments()
        ctx.solver, ctx.nsteps, ctx.every = solver, nsteps, every
        ctx.checkpoints, ctx.tail, ctx.final_state = checkpoints, tail, final_state
        ctx.save_for_backward(n0.detach(), ux0.detach(), uy0.detach(), T0.detach())
        return n, ux, uy, T

    @staticmethod
    def backward(ctx, gn, gux, guy, gT):
        s = ctx.solver
        n0, ux0, uy0, T0 = ctx.saved_tensors
        g = [x if x is not None else _zeros_like_field(s) for x in (gn, gux, guy, gT)]
        lam = s.moments_adjoint(ctx.final_state, *g)
        main = torch.cuda.current_stream(s.device)
        every, nsteps = ctx.every, ctx.nsteps
        nseg = len(ctx.checkpoints) + (1 if ctx.tail is not None else 0)
        # recomputing one segment ahead on a second stream keeps up to three
        # segments alive (the one the adjoint walks, the one being recomputed,
        # and the previous one until the caller's stream has released it);
        # without room for two more, every segment is recomputed on the
        # caller's stream just before its adjoint
        ahead = nseg > 1 and _memory_budget(s) >= 2 * _segment_bytes(s, min(every, nsteps))
        side = s.side_stream() if ahead else None

        def recompute(seg):
            start = seg * every
            count = min(start + every, nsteps) - start
            ck = ctx.checkpoints[seg]
            if side is None:
                s.bind_state(ck)  # read only by the out-of-place steps
                states, records = _recorded_segment(s, count)
                return states, records, None
            # starts once the caller's stream has finished what it was given
            # so far (at most one segment is recomputed ahead of the adjoint)
            side.wait_stream(main)
            with torch.cuda.stream(side):
                s.set_stream(side)
                ck.record_stream(side)
                s.bind_state(ck)
                states, records = _recorded_segment(s, count)
                ev = torch.cuda.Event()
                ev.record(side)
            s.set_stream(main)
            for t in states[1:] + records:
                t.record_stream(main)
            return states, records, ev

        try:
            pending = None
            if nseg:
                pending = (*ctx.tail, None) if ctx.tail is not None else recompute(nseg - 1)
            for seg in reversed(range(nseg)):
                states, records, ev = pending
                pending = None
                if ev is not None:
                    main.wait_event(ev)
                if ahead and seg > 0:
                    pending = recompute(seg - 1)
                F = rec = None
                for F, rec in zip(reversed(states), reversed(records)):
                    lam = s.adjoint_step(F, lam, record=rec)
                del states, records, F, rec
                if seg == nseg - 1:
                    ctx.tail = None  # the forward's records of the last segment are done with
                if not ahead and seg > 0:
                    pending = recompute(seg - 1)
        finally:
            s.set_stream(main)  # also when a call above raised
        if side is not None:
            s.state.record_stream(main)
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
