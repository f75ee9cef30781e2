"""torch.autograd wrappers over the hand-written adjoints in libttc.so.

TTInner: z = <X, Y> with gradients for every core of X and Y (adjoint
sweeps that keep every c-th interface and recompute the rest).
TTLinear: y = W x for a TT-matrix W, gradients for the input batch and every
core.  Both save only their inputs, except TTLinear with the schedule
"cores_saved", which also keeps the forward's workspace (its per-core
intermediates) for the backward."""
from __future__ import annotations

import torch

from . import api


class TTInner(torch.autograd.Function):
    @staticmethod
    def forward(ctx, n_x: int, ckpt_stride: int, *cores):
        x, y = list(cores[:n_x]), list(cores[n_x:])
        ctx.n_x = n_x
        ctx.ckpt_stride = ckpt_stride
        ctx.save_for_backward(*cores)
        return api.tt_contract_inner(x, y)

    @staticmethod
    def backward(ctx, gz):
        cores = ctx.saved_tensors
        x, y = list(cores[:ctx.n_x]), list(cores[ctx.n_x:])
        nx = any(ctx.needs_input_grad[2:2 + ctx.n_x])
        ny = any(ctx.needs_input_grad[2 + ctx.n_x:])
        gx, gy = api.tt_contract_inner_bwd(x, y, gz.detach(), ckpt_stride=ctx.ckpt_stride, need_x=nx, need_y=ny)
        gx = [g.to(c.dtype) for g, c in zip(gx, x)] if gx is not None else [None] * len(x)
        gy = [g.to(c.dtype) for g, c in zip(gy, y)] if gy is not None else [None] * len(y)
        return (None, None, *gx, *gy)


def tt_inner(x, y, ckpt_stride: int = 0):
    return TTInner.apply(len(x), ckpt_stride, *x, *y)


class TTLinear(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, prec: str, sched: str, *cores):
        ctx.prec, ctx.sched = prec, sched
        ctx.save_for_backward(x, *cores)
        ctx.ws = None
        if sched == "cores_saved":
            need = api.ttm_apply_dense_query(list(cores), x.shape[0], prec, sched, backward=True)
            ctx.ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
        return api.ttm_apply_dense(list(cores), x, prec=prec, sched=sched, ws=ctx.ws)

    @staticmethod
    def backward(ctx, dy):
        x, *cores = ctx.saved_tensors
        dx, dcores = api.ttm_apply_dense_bwd(list(cores), x, dy.contiguous(), prec=ctx.prec, sched=ctx.sched,
                                             need_dx=ctx.needs_input_grad[0],
                                             need_dw=any(ctx.needs_input_grad[3:]), ws=ctx.ws)
        ctx.ws = None
        if dcores is None:
            dcores = [None] * len(cores)
        return (dx, None, None, *dcores)


def tt_linear(x, cores, prec: str = "auto", sched: str = "auto"):
    return TTLinear.apply(x, prec, sched, *cores)
