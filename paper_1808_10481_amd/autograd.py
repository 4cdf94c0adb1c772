"""torch.autograd wrapper of the Hermite-leapfrog step (argument marshalling
only: the forward runs hl_step, the backward hl_adjoint_step).

The n-step map (P, U) -> (P_n, U_n) is linear in the state, so its
vector-Jacobian product with respect to the state is the discrete adjoint
applied to the incoming gradients.  The derivative with respect to kappa = c^2
(dt held fixed) comes from the same call, which walks the forward state back
with the reversed step.  Tensors are the plan's device state buffers (periodic
plans, FP64 or FP32).
"""

from __future__ import annotations

import torch


class HermiteSteps(torch.autograd.Function):
    """(p, u, kappa) -> (p_n, u_n) after `nsteps` steps of `plan` (an hl.Plan).
    `kappa` is a 0-d FP64 tensor equal to the plan's kappa; it only carries
    the gradient with respect to the coefficient."""

    @staticmethod
    def forward(ctx, p, u, kappa, plan, nsteps):
        if abs(float(kappa) - plan.kappa) > 1e-12 * plan.kappa:
            raise ValueError("kappa differs from the plan's kappa; build a plan for it")
        ctx.plan, ctx.nsteps = plan, int(nsteps)
        p_n, u_n = p.detach().clone(), u.detach().clone()
        plan.step(p_n, u_n, ctx.nsteps)
        ctx.save_for_backward(p_n, u_n)
        return p_n, u_n

    @staticmethod
    def backward(ctx, g_p, g_u):
        plan = ctx.plan
        p_n, u_n = ctx.saved_tensors
        pb = g_p.detach().contiguous().clone() if g_p is not None else torch.zeros_like(p_n)
        ub = g_u.detach().contiguous().clone() if g_u is not None else torch.zeros_like(u_n)
        gk = None
        if ctx.needs_input_grad[2]:
            gk = torch.zeros(1, dtype=torch.float64, device=p_n.device)
            plan.adjoint_step(pb, ub, ctx.nsteps, p=p_n, u=u_n, grad_kappa=gk)
            gk = gk.reshape(())
        else:
            plan.adjoint_step(pb, ub, ctx.nsteps)
        return pb, ub, gk, None, None


def hermite_steps(p, u, plan, nsteps, kappa=None):
    """(p_n, u_n) = nsteps steps of plan from (p, u), differentiable in p, u
    and (when given as a tensor) kappa."""
    if kappa is None:
        kappa = torch.tensor(plan.kappa, dtype=torch.float64)
    return HermiteSteps.apply(p, u, kappa, plan, nsteps)
