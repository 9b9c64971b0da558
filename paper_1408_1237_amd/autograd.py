"""Differentiable kernel solve: w = (K_hat(x; sigma) + gamma I)^{-1} y.

Forward: the mixed-precision flexible GMRES of the library.  Backward: one
adjoint solve lambda = K^{-1} (dl/dw) with the same solver (K is symmetric)
and one gradient pass (kmvp_grad) giving dl/dx, dl/dlog sigma and dl/dlog gamma;
dl/dy = lambda.  Hyperparameters are estimated by maximum likelihood in the
paper's GPR experiments (section 2.1, section 6.1); this gives the gradients
that such an estimation needs.
"""
from __future__ import annotations

import math

import torch

from . import api


class KrrSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, y, log_sigma, log_gamma, opts):
        sigma = math.exp(float(log_sigma))
        gamma = math.exp(float(log_gamma))
        opts = dict(opts or {})
        grad_prec = opts.pop("grad_prec", "fp64")
        w, info = api.fgmres_solve(x.detach().contiguous(), sigma, gamma, y.detach().contiguous(), **opts)
        if info["status"] != 0:
            raise RuntimeError(f"forward solve did not converge: {info}")
        ctx.save_for_backward(x, w)
        ctx.sigma, ctx.gamma, ctx.opts, ctx.grad_prec = sigma, gamma, opts, grad_prec
        ctx.shapes = (log_sigma.shape, log_gamma.shape)
        return w

    @staticmethod
    def backward(ctx, gw):
        x, w = ctx.saved_tensors
        lam, info = api.fgmres_solve(x.detach().contiguous(), ctx.sigma, ctx.gamma, gw.contiguous(), **ctx.opts)
        if info["status"] != 0:
            raise RuntimeError(f"adjoint solve did not converge: {info}")
        gx, gls, glg = api.kmvp_grad(x.detach().contiguous(), ctx.sigma, ctx.gamma, lam, w, prec=ctx.grad_prec)
        s_shape, g_shape = ctx.shapes
        return gx, lam, gls.reshape(s_shape), glg.reshape(g_shape), None


def krr_solve(x, y, log_sigma, log_gamma, **opts):
    """w = (K_hat + gamma I)^{-1} y, differentiable in x, y, log_sigma and log_gamma.

    opts: the solver options of fgmres_solve (used by the forward and the adjoint
    solve) and grad_prec ("fp64" default, or "fp32") for the gradient pass."""
    return KrrSolve.apply(x, y, log_sigma, log_gamma, opts)
