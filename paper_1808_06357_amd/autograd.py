"""torch.autograd.Function over strang_run / strang_adjoint.

Forward: m Strang steps of eq. (StrangTDSE) from u0 under v (checkpoints are
stored every `ckpt_every` steps).  Backward: the hand-written adjoint kernel
(reverse-time recomputation reset at the checkpoints) gives dJ/du0 and dJ/dv.
Complex gradients follow torch's convention dJ/dRe + i dJ/dIm.
"""
from __future__ import annotations

import torch

from . import _capi


class LatticeStrang(torch.autograd.Function):
    @staticmethod
    def forward(ctx, v, u0, plan, gamma, dt, steps, ckpt_every):
        N = plan.N
        batch = u0.numel() // N
        u = u0.detach().clone().contiguous()
        v = v.detach().contiguous()
        nck = _capi.num_checkpoints(steps, ckpt_every)
        ckpt = torch.empty(max(nck, 1) * batch * N, dtype=u.dtype, device=u.device)
        _capi.strang_run(plan, v, u, gamma, dt, steps, ckpt=ckpt if nck else None,
                         ckpt_every=ckpt_every if nck else 0)
        ctx.plan, ctx.gamma, ctx.dt, ctx.steps, ctx.every = plan, gamma, dt, steps, ckpt_every
        ctx.save_for_backward(v, u, ckpt)
        return u.view_as(u0)

    @staticmethod
    def backward(ctx, grad_u):
        v, uT, ckpt = ctx.saved_tensors
        gT = grad_u.contiguous().to(uT.dtype)
        g0, gv = _capi.strang_adjoint(ctx.plan, v, uT, gT, ctx.gamma, ctx.dt, ctx.steps,
                                      ckpt if ctx.steps else None, ctx.every)
        return gv.view_as(v), g0.view_as(grad_u), None, None, None, None, None


def lattice_strang(plan, v, u0, gamma: float, dt: float, steps: int, ckpt_every: int = 50):
    """Differentiable u(T) = S^m u0 (S the Strang step on plan's lattice)."""
    return LatticeStrang.apply(v, u0, plan, gamma, dt, steps, ckpt_every)
