"""The differentiable unrolled RTCUR-F behind torch.autograd.

    plan = rt.unroll_plan(dims, ranks, I_sizes, K=15, seed=0)
    L = UnrolledRTCUR.apply(X, zetas, plan, tau)   # L^K on the sampled blocks
    loss(L).backward()                              # zetas.grad, X.grad

Forward and backward are the library's kernels (rtcur_unroll_forward,
rtcur_unroll_backward): this module only hands tensors across.  One plan
holds the checkpoints of one forward pass, so each forward is followed by
its own backward before the plan's next forward.
"""

from __future__ import annotations

import torch

from . import unroll_backward, unroll_forward


class UnrolledRTCUR(torch.autograd.Function):
    """X (device, float32/float64, the plan's dims), zetas (K thresholds, a
    tensor that may require grad), plan (UnrollPlan), tau (gate temperature;
    0: the hard threshold, whose zeta-gradient is zero).  Returns L^K on the
    sampled blocks, float64 on X's device."""

    @staticmethod
    def forward(ctx, X, zetas, plan, tau):
        L = unroll_forward(plan, X.detach(), zetas.detach(), float(tau))
        ctx.plan = plan
        ctx.generation = plan.generation
        ctx.x_dtype = X.dtype
        ctx.z_meta = (zetas.dtype, zetas.device)
        return L

    @staticmethod
    def backward(ctx, L_bar):
        plan = ctx.plan
        if plan.generation != ctx.generation:
            raise RuntimeError("the plan ran another forward pass before this backward")
        zb, Xb = unroll_backward(plan, L_bar)
        dz = torch.from_numpy(zb).to(dtype=ctx.z_meta[0], device=ctx.z_meta[1])
        return Xb.to(ctx.x_dtype), dz, None, None
