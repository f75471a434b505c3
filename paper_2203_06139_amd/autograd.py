"""The histogram objective as a differentiable torch function.

L(theta, w) = sum_i w_i l(n_i, mu_i(theta)).  Forward calls nll_eval; backward
is the reverse-mode adjoint kernel (nll_grad) seeded with the upstream
gradient, which stays on the device and is read by the kernel through a
pointer (no host synchronisation).  It returns dL/dtheta * seed and, when the
weights require a gradient, dL/dw_i * seed = l_i * seed per bin.  This is
reverse accumulation as the paper motivates it (sec. 2: one output, many
inputs, gradient cost independent of the number of inputs), with the bins'
weights as the "many inputs".
"""
from __future__ import annotations

import torch
from torch.autograd.function import once_differentiable

from . import FP64, POISSON, Hist, Model, nll_eval, nll_grad


class HistNLL(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta, weights, counts, xrange, yrange, model, objective, precision, edges):
        hist = Hist(counts, tuple(xrange), tuple(yrange), weights, edges)
        out = nll_eval(hist, model, theta, objective=objective, precision=precision)
        ctx.save_for_backward(theta, weights, counts, edges)
        ctx.meta = (tuple(xrange), tuple(yrange), model, objective, precision)
        return out.reshape(())

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        theta, weights, counts, edges = ctx.saved_tensors
        xrange, yrange, model, objective, precision = ctx.meta
        hist = Hist(counts, xrange, yrange, weights, edges)
        seed = g.detach().to(torch.float64).reshape(1).contiguous()
        want_w = weights is not None and ctx.needs_input_grad[1]
        _, grad, gw = nll_grad(hist, model, theta, objective=objective, precision=precision,
                               seed=seed, want_grad_w=want_w)
        grad_theta = grad if ctx.needs_input_grad[0] else None
        grad_w = gw.reshape(weights.shape) if want_w else None
        return grad_theta, grad_w, None, None, None, None, None, None, None


def hist_nll(theta: torch.Tensor, counts: torch.Tensor, model: Model, xrange, yrange=(0.0, 1.0),
             weights: torch.Tensor | None = None, objective: int = POISSON,
             precision: int = FP64, edges: torch.Tensor | None = None) -> torch.Tensor:
    """Differentiable L(theta, w) for device tensors: theta f64[P], counts
    [nx] or [ny, nx] (int32 read as u32, f32 or f64), weights f32 of the same
    shape or None; edges (1D, f64[nx + 1] ascending, not differentiated) for
    bins of any widths."""
    if theta.dtype != torch.float64:
        raise TypeError("theta must be float64")
    if weights is not None and weights.dtype != torch.float32:
        raise TypeError("weights must be float32")
    if edges is not None and (edges.dtype != torch.float64 or edges.numel() != counts.numel() + 1):
        raise ValueError("edges must be f64 with nx + 1 values")
    return HistNLL.apply(theta, weights, counts, xrange, yrange, model, objective, precision,
                         edges)
