"""torch.autograd.Function wrappers of the space-time operators.

Each operator's backward is the library's hand-written adjoint kernel:

    ForwardOp   b = H u                 du = H^T gb
    GradientOp  (gx, gy) = Psi u        du = Psi^T (ggx, ggy)
    FlowOp      r = L(v) u              du = L(v)^T gr,   dv = (d(L(v)u)/dv)^T gr

so a loss built from several of them gets its gradient from the adjoint kernels, with
autograd adding the contributions of the operators that share an input.  Tensors are
flat, contiguous GPU tensors in the layouts of the C ABI (frames [t][y][x], flows
[pair][2][y][x]).
"""
from __future__ import annotations

import torch

from . import _lib
from . import binding as B


class ForwardOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, plan):
        ctx.plan = plan
        return B.apply_A(plan, u.contiguous())

    @staticmethod
    def backward(ctx, gb):
        return B.apply_At(ctx.plan, gb.contiguous()), None


class GradientOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, stack):
        ctx.stack = stack
        return B.apply_grad(stack, u.contiguous())

    @staticmethod
    def backward(ctx, ggx, ggy):
        # autograd materialises an unused output's gradient as zeros
        return B.apply_grad(ctx.stack, gx=ggx.contiguous(), gy=ggy.contiguous(), transpose=True), None


class FlowOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, u, v, stack, direction, interp):
        u = u.contiguous()
        v = v.contiguous()
        ctx.save_for_backward(u, v)
        ctx.stack, ctx.direction, ctx.interp = stack, direction, interp
        return B.apply_flow_op(stack, _lib.MMOF_FLOW_FWD, direction, interp, u, v)

    @staticmethod
    def backward(ctx, gr):
        u, v = ctx.saved_tensors
        gr = gr.contiguous()
        du = dv = None
        if ctx.needs_input_grad[0]:
            du = B.apply_flow_op(ctx.stack, _lib.MMOF_FLOW_ADJ, ctx.direction, ctx.interp, None, v, gr)
        if ctx.needs_input_grad[1]:
            dv = B.apply_flow_op(ctx.stack, _lib.MMOF_FLOW_DV, ctx.direction, ctx.interp, u, v, gr)
        return du, dv, None, None, None


def forward_op(u, plan):
    """H u with gradient H^T."""
    return ForwardOp.apply(u, plan)


def gradient_op(u, stack):
    """(gx, gy) = Psi u with gradient Psi^T."""
    return GradientOp.apply(u, stack)


def flow_op(u, v, stack, direction: int = 1, interp: int = _lib.MMOF_INTERP_BILINEAR):
    """L(v) u with gradients L(v)^T (for u) and the bilinear-warp derivative (for v)."""
    return FlowOp.apply(u, v, stack, direction, interp)
