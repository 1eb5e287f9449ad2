"""Differentiable unrolled A-MMMSE: a torch.autograd.Function over the
library's ammse_unrolled_forward / ammse_unrolled_backward (hand-written
adjoint kernels; checkpoints every `ckpt_every` iterations).

    wsr = unrolled_wsr(plan, db, gamma, H=None, ckpt_every=5)

`gamma` is a [B, T] (or [T], shared by the batch) real tensor of step sizes
on the device; `H` defaults to the batch's channels and may require grad
(complex, the library's flat layout).  The result is WSR(V^T) per instance;
its gradient flows to gamma and H (torch's complex convention:
dL = Re sum(conj(H.grad) * dH)).  The stage switch and the projection
branch of the forward are held fixed in the backward.
"""
from typing import Optional

import torch

from . import ammse


class _Unrolled(torch.autograd.Function):
    @staticmethod
    def forward(ctx, gamma, H, plan, db, ckpt_every, force_switch):
        B, T = gamma.shape
        dev = gamma.device
        ws_bytes, ck_bytes = plan.unrolled_sizes(ckpt_every)
        ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
        ck = torch.empty(ck_bytes, dtype=torch.uint8, device=dev)
        V = db.V0.clone()
        wsr = torch.empty(B, dtype=torch.float64, device=dev)
        sw = torch.empty(B, dtype=torch.int32, device=dev)
        st = torch.empty(B, dtype=torch.int32, device=dev)
        g = gamma.detach().to(torch.float64).contiguous()
        Hd = H.detach().contiguous()
        plan.unrolled_forward(Hd, db.sigma2, db.alpha, db.P, V, g, ckpt_every, wsr, sw, ck, ws,
                              status=st, force_switch=force_switch)
        ctx.save_for_backward(g, Hd)
        ctx.plan, ctx.db, ctx.ck, ctx.ws, ctx.sw, ctx.K = plan, db, ck, ws, sw, ckpt_every
        ctx.gamma_dtype = gamma.dtype
        ctx.mark_non_differentiable(V, sw, st)
        return wsr, V, sw, st

    @staticmethod
    def backward(ctx, gwsr, gV, gsw, gst):
        if gV is not None and bool(torch.any(gV != 0)):
            raise NotImplementedError("gradients flow from WSR(V^T) only")
        g, Hd = ctx.saved_tensors
        dH = torch.empty_like(Hd)
        dg = torch.empty_like(g)
        dw = (gwsr if gwsr is not None else torch.zeros_like(g[:, 0])).to(torch.float64).contiguous()
        db = ctx.db
        ctx.plan.unrolled_backward(Hd, db.sigma2, db.alpha, db.P, g, ctx.K, ctx.sw, ctx.ck, dw,
                                   dH, dg, ctx.ws)
        return dg.to(ctx.gamma_dtype), dH, None, None, None, None


def unrolled_wsr(plan: "ammse.Plan", db: "ammse.DeviceBatch", gamma: torch.Tensor,
                 H: Optional[torch.Tensor] = None, ckpt_every: int = 5,
                 force_switch: Optional[torch.Tensor] = None):
    """WSR(V^T) per instance (differentiable in gamma and H), plus V^T, the
    switch iterations and the status flags (not differentiable)."""
    B = plan.batch
    if gamma.dim() == 1:
        gamma = gamma.unsqueeze(0).expand(B, -1)
    if gamma.shape[1] != plan.options.max_iters:
        raise ValueError("gamma must hold one step size per iteration")
    if H is None:
        H = db.H
    return _Unrolled.apply(gamma, H, plan, db, int(ckpt_every), force_switch)
