"""torch.autograd wrappers: gridding and degridding are each other's adjoints.

For one plan, degridding is the linear map D with real coefficients (the product
of the two sampled kernel rows), and gridding with weights w is D^T diag(w), so
the backward pass of each is a call of the other:

  * DegridFn: M = D G;            dL/dG = D^T dL/dM        (rts_grid with w = 1)
  * GridFn:   G = D^T (w V);      dL/dV = w D(dL/dG),  dL/dw = Re(conj(V) D(dL/dG))
                                  (rts_grid_backward)
  * Chi2Fn:   L = sum w |V - D G|^2 over valid samples, from one fused pass
              (rts_grid_degrid); dL/dG = -2 D^T(w r), dL/dw = |r|^2, dL/dV = 2 w r
              (rts_chi2_backward, from the fused pass's model and grid)

Gradients follow PyTorch's convention for complex tensors (dL/dRe + i dL/dIm).
The products, the residual and the element-wise gradient terms all run in the
library's HIP kernels; these classes route tensors and allocate the outputs.
Plans built with conjugate copies are rejected: their gridding also adds
conj(w V) at -uv, which is not complex-linear in V, and their degridding
predicts the +uv copy only.
"""
from __future__ import annotations

import torch


def _linear_plan(plan):
    if plan.params.conjugate:
        raise ValueError("autograd needs a plan without conjugate copies (conjugate=False)")
    return plan


class DegridFn(torch.autograd.Function):
    """M = degrid(G) for a plan; backward grids the incoming gradient with unit weights."""

    @staticmethod
    def forward(ctx, G, plan):
        ctx.plan = _linear_plan(plan)
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
        ctx.plan = _linear_plan(plan)
        ctx.save_for_backward(V, w)
        return plan.grid(V.contiguous(), w.contiguous())

    @staticmethod
    def backward(ctx, gG):
        V, w = ctx.saved_tensors
        gV, gw = ctx.plan.grid_backward(V.contiguous(), w.contiguous(), gG.contiguous(),
                                        want_weights=ctx.needs_input_grad[1])
        return (gV if ctx.needs_input_grad[0] else None), gw, None


class Chi2Fn(torch.autograd.Function):
    """chi2 = sum_i w_i |V_i - degrid(G)_i|^2 over valid samples (FP64 scalar).

    The forward is one fused pass that also grids the weighted residual, which is
    exactly the gradient with respect to G up to the factor -2; the backward forms
    the three gradients from that grid and the model in one library call."""

    @staticmethod
    def forward(ctx, V, w, G, plan):
        ctx.plan = _linear_plan(plan)
        V, w = V.contiguous(), w.contiguous()
        model, g_out, chi2 = plan.grid_degrid(V, w, G.contiguous())
        ctx.save_for_backward(V, w, model, g_out)
        return chi2

    @staticmethod
    def backward(ctx, g):
        V, w, model, g_out = ctx.saved_tensors
        g = g.to(torch.float64).contiguous()
        gV, gw, gG = ctx.plan.chi2_backward(V, w, model, g_out, g, want=tuple(ctx.needs_input_grad[:3]))
        return gV, gw, gG, None


def grid(V, w, plan):
    return GridFn.apply(V, w, plan)


def degrid(G, plan):
    return DegridFn.apply(G, plan)


def chi2(V, w, G, plan):
    return Chi2Fn.apply(V, w, G, plan)
