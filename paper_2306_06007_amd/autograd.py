"""Differentiation through HVOX synthesis.

``HvoxSynthesis.apply(x, plan)`` returns V = A x (sky -> vis).  Its backward
is the hand-written analysis kernel: for complex x the gradient is A^H g
(PyTorch passes the conjugate-Wirtinger gradient g of a real loss with
respect to V); for real x it is Re(A^H g), the real-valued adjoint the paper
enforces for sky intensity maps (Sect. 4, the `real` option)."""
from __future__ import annotations

import torch


class HvoxSynthesis(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        ctx.real_input = not x.is_complex()
        ctx.in_dtype = x.dtype
        xc = x.to(plan.complex_dtype) if ctx.real_input else x
        return plan.synthesis(xc)

    @staticmethod
    def backward(ctx, g):
        gx = ctx.plan.analysis(g.contiguous())
        if ctx.real_input:
            gx = gx.real.to(ctx.in_dtype)
        return gx, None


class HvoxAnalysis(torch.autograd.Function):
    """I = A^H V with backward A g (synthesis)."""

    @staticmethod
    def forward(ctx, v, plan):
        ctx.plan = plan
        return plan.analysis(v)

    @staticmethod
    def backward(ctx, g):
        return ctx.plan.synthesis(g.contiguous()), None


def synthesis(x, plan):
    return HvoxSynthesis.apply(x, plan)


def analysis(v, plan):
    return HvoxAnalysis.apply(v, plan)
