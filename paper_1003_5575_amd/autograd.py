"""torch.autograd wrappers: gridding and degridding are each other's adjoints.

For one plan, degridding is the linear map D with real coefficients (the product
of the two sampled kernel rows), and gridding with weights w is D^T diag(w), so
the backward pass of each is a call of the other:

  * DegridFn: M = D G;            dL/dG = D^T dL/dM        (rts_grid with w = 1)
  * GridFn:   G = D^T (w V);      dL/dV = w D(dL/dG),  dL/dw = Re(conj(V) D(dL/dG))
  * Chi2Fn:   L = sum w |V - D G|^2 over valid samples, from one fused pass
              (rts_grid_degrid); dL/dG = -2 D^T(w r), dL/dw = |r|^2, dL/dV = 2 w r

Gradients follow PyTorch's convention for complex tensors (dL/dRe + i dL/dIm).
Every product runs in the library's HIP kernels; these classes only route
tensors.
"""
from __future__ import annotations

import torch


class DegridFn(torch.autograd.Function):
    """M = degrid(G) for a plan; backward grids the incoming gradient with unit weights."""

    @staticmethod
    def forward(ctx, G, plan):
        ctx.plan = plan
        return plan.degrid(G.contiguous())

    @staticmethod
    def backward(ctx, gM):
        plan = ctx.plan
        ones = torch.ones((plan.C, plan.B, plan.T), dtype=torch.float32, device=gM.device)
        return plan.grid(gM.contiguous(), ones), None


class GridFn(torch.autograd.Function):
    """G = grid(V, w) for a plan; backward degrids the incoming gradient once."""

    @staticmethod
    def forward(ctx, V, w, plan):
        ctx.plan = plan
        ctx.save_for_backward(V, w)
        return plan.grid(V.contiguous(), w.contiguous())

    @staticmethod
    def backward(ctx, gG):
        V, w = ctx.saved_tensors
        d = ctx.plan.degrid(gG.contiguous())          # 0 at invalid samples
        gV = gw = None
        if ctx.needs_input_grad[0]:
            gV = d * w
        if ctx.needs_input_grad[1]:
            gw = (torch.conj(V) * d).real
        return gV, gw, None


class Chi2Fn(torch.autograd.Function):
    """chi2 = sum_i w_i |V_i - degrid(G)_i|^2 over valid samples (FP64 scalar).

    The forward is one fused pass that also grids the weighted residual, which is
    exactly the gradient with respect to G; the backward only scales it."""

    @staticmethod
    def forward(ctx, V, w, G, plan):
        model, g_out, chi2 = plan.grid_degrid(V.contiguous(), w.contiguous(), G.contiguous())
        # residual in place of the model (a buffer of this call): V - M, 0 where invalid
        r = torch.sub(V, model, out=model)
        r.masked_fill_(~plan.valid_mask(), 0)
        ctx.save_for_backward(r, w, g_out)
        return chi2

    @staticmethod
    def backward(ctx, g):
        r, w, g_out = ctx.saved_tensors
        g32 = g.to(torch.float32)
        gV = gw = gG = None
        if ctx.needs_input_grad[0]:
            gV = (2.0 * g32) * w * r
        if ctx.needs_input_grad[1]:
            gw = torch.view_as_real(r).square().sum(-1).mul_(g32)
        if ctx.needs_input_grad[2]:
            gG = g_out * (-2.0 * g32)
        return gV, gw, gG, None


def grid(V, w, plan):
    return GridFn.apply(V, w, plan)


def degrid(G, plan):
    return DegridFn.apply(G, plan)


def chi2(V, w, G, plan):
    return Chi2Fn.apply(V, w, G, plan)
