"""Differentiable cycle-averaged eddy-current loss.

eddy_loss(problem, theta_cell, sigma_cell) returns the Joule loss of one period,
    l = tau sum_n (d u^n)^T M (d u^n),  d u^n = (u^n - u^{n-1}) / tau,
of the periodic solution U of Problem 1 for the given per-cell reluctivity scale theta
(nu = theta nuhat) and per-cell conductivity sigma (each cell's two triangles share
its value). It is a torch.autograd.Function: the forward pass runs the fixed-point
solve (pt_solve) and keeps the converged iterate U as the checkpoint of the backward
pass; the backward pass solves the adjoint system J^T lambda = dl/dU, which runs
backward in time and is periodic (pt_adjoint_solve), and forms the per-cell gradients
(pt_loss_gradients). Because U is a fixed point, the gradient needs only U (implicit
differentiation), not the iterates that led to it.

Only argument marshalling happens here; every step runs in the HIP library.
"""
from __future__ import annotations

import dataclasses

from . import Plan


def _make():
    import torch

    class EddyLoss(torch.autograd.Function):
        @staticmethod
        def forward(ctx, theta_cell, sigma_cell, problem, opts):
            theta_t = theta_cell.detach().repeat_interleave(2).contiguous()
            sigma_t = sigma_cell.detach().repeat_interleave(2).contiguous()
            plan = Plan(problem, theta=theta_t, sigma=sigma_t, adjoint=True, **opts)
            U, st = plan.solve()
            loss, _, _ = plan.loss_gradients(U, None)
            ctx.plan = plan
            ctx.keep = (theta_t, sigma_t)
            ctx.save_for_backward(U)
            ctx.stats = st
            return torch.tensor(loss, dtype=torch.float64, device=theta_cell.device)

        @staticmethod
        def backward(ctx, grad_out):
            (U,) = ctx.saved_tensors
            plan = ctx.plan
            Lam, ast = plan.adjoint_solve(U)
            _, gt, gs = plan.loss_gradients(U, Lam, per_cell=True)
            ctx.adjoint_stats = ast
            g = grad_out.to(gt.dtype)
            plan.close()
            return g * gt, g * gs, None, None

    return EddyLoss


_fn = None


def eddy_loss(problem, theta_cell, sigma_cell, **opts):
    """Loss of the periodic solution for per-cell theta and sigma (float64 device tensors of
    n^2 entries, cell id j n + i); differentiable in both. opts go to Plan (tol, precision,
    max_outer, ...). The problem's own theta field is ignored."""
    global _fn
    if _fn is None:
        _fn = _make()
    problem = dataclasses.replace(problem, theta=None)
    return _fn.apply(theta_cell, sigma_cell, problem, opts)
