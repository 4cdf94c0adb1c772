"""torch.autograd wrappers of the Hermite-leapfrog step (argument marshalling
only: the forward runs hl_step, the backward hl_adjoint_step, or
hl_adjoint_step_var for variable kappa).

The n-step map (P, U) -> (P_n, U_n) is linear in the state, so its
vector-Jacobian product with respect to the state is the discrete adjoint
applied to the incoming gradients.  The derivative with respect to kappa = c^2
(dt held fixed) comes from the same call, which walks the forward state back
with the reversed step.  Tensors are the plan's device state buffers (FP64 or
FP32; periodic or walled plans).
"""

from __future__ import annotations

import numpy as np
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


# ---------------------------------------------------------------------------
# Variable kappa: receiver traces and their gradient with respect to the kappa
# data, with sqrt(N) checkpointing.
# ---------------------------------------------------------------------------

def receiver_index(plan, receivers):
    """Device word index of coefficient 0 of the pressure at each receiver
    (host node tuples (j_1, .., j_d) of the primal nodes: K per dimension, or
    K+1 with walls): the p layout stores plane 0 first, nodes with j_1
    fastest."""
    ext = plan.host_shapes()[0][:plan.d]
    idx = []
    for r in receivers:
        n, stride = 0, 1
        for k, j in enumerate(r):
            if not 0 <= int(j) < ext[k]:
                raise ValueError(f"receiver {r} outside the primal nodes {ext}")
            n += int(j) * stride
            stride *= ext[k]
        idx.append(n)
    return torch.tensor(idx, dtype=torch.int64, device="cuda")


class ReceiverTraces(torch.autograd.Function):
    """(kappa_p, kappa_u, p, u) -> (traces, p_n, u_n): nsteps variable-kappa
    steps of `plan` from (p, u) with kappa data kappa_p, kappa_u (FP64 CPU
    tensors in hl_set_kappa's layout); traces[t, r] is coefficient 0 of the
    pressure at receiver r after step t + 1.

    The forward keeps the state every `seg` steps (seg = ceil(sqrt(nsteps))
    by default); the backward re-runs each segment from its checkpoint, last
    segment first, and undoes its steps one by one with hl_adjoint_step_var,
    adding the traces' gradient at the receivers to p_bar before undoing the
    step that produced them.  Memory: about 2 sqrt(nsteps) states.  Reading
    the traces and adding their gradient are plain index operations on the
    state (observation, not part of the step)."""

    @staticmethod
    def forward(ctx, kappa_p, kappa_u, p, u, plan, nsteps, rec_index, seg):
        nsteps = int(nsteps)
        seg = int(seg) if seg else max(1, int(np.ceil(np.sqrt(nsteps))))
        plan.set_kappa(kappa_p.detach().cpu().numpy(), kappa_u.detach().cpu().numpy())
        p_n, u_n = p.detach().clone(), u.detach().clone()
        traces = torch.empty((nsteps, rec_index.numel()), dtype=p.dtype, device=p.device)
        ckpts = []
        for t in range(nsteps):
            if t % seg == 0:
                ckpts.append((p_n.clone(), u_n.clone()))
            plan.step(p_n, u_n, 1)
            traces[t] = p_n[rec_index]
        ctx.plan, ctx.nsteps, ctx.seg, ctx.rec, ctx.ckpts = plan, nsteps, seg, rec_index, ckpts
        ctx.kappa_shape = (tuple(kappa_p.shape), tuple(kappa_u.shape))
        return traces, p_n, u_n

    @staticmethod
    def backward(ctx, g_tr, g_p, g_u):
        plan, nsteps, seg, rec = ctx.plan, ctx.nsteps, ctx.seg, ctx.rec
        p0, u0 = ctx.ckpts[0]
        pb = g_p.detach().contiguous().clone() if g_p is not None else torch.zeros_like(p0)
        ub = g_u.detach().contiguous().clone() if g_u is not None else torch.zeros_like(u0)
        g_tr = g_tr.detach().to(pb.dtype) if g_tr is not None else None
        plan.kappa_grad(reset=True)  # start from zero
        for c in range(len(ctx.ckpts) - 1, -1, -1):
            t0 = c * seg
            t1 = min(nsteps, t0 + seg)
            ps, us = [ctx.ckpts[c][0].clone()], [ctx.ckpts[c][1].clone()]
            for _ in range(t0, t1):
                pn, un = ps[-1].clone(), us[-1].clone()
                plan.step(pn, un, 1)
                ps.append(pn)
                us.append(un)
            for t in range(t1 - 1, t0 - 1, -1):
                if g_tr is not None:
                    pb.index_add_(0, rec, g_tr[t])
                plan.adjoint_step_var(pb, ub, ps[t + 1 - t0], us[t - t0])
        gkp, gku = plan.kappa_grad(reset=True)
        return (torch.from_numpy(gkp).reshape(ctx.kappa_shape[0]), torch.from_numpy(gku).reshape(ctx.kappa_shape[1]),
                pb, ub, None, None, None, None)


def receiver_traces(kappa_p, kappa_u, p, u, plan, nsteps, receivers, seg=None):
    """Differentiable receiver traces (see ReceiverTraces); receivers are host
    node tuples."""
    return ReceiverTraces.apply(kappa_p, kappa_u, p, u, plan, nsteps, receiver_index(plan, receivers), seg)
