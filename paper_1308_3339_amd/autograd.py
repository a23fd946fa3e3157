"""torch.autograd wrappers of the solve and of the Gaussian-bump source.

``poisson_solve(plan, f)`` returns u = A^{-1} f through the FMM-preconditioned
FGMRES of the library; its backward runs the adjoint solve
(``precond_gmres_solve_adjoint``: A^T lambda = dL/du, A^T = A for the 5-point
matrix), so dL/df = lambda.  ``gaussian_bumps(plan, cx, cy, w, a)`` evaluates
the bump source on the plan's grid (``fmm_bumps_eval``); its backward carries
dL/df to the bump parameters (``fmm_bumps_grad``).  Both run entirely in the
library's kernels; torch supplies memory, streams and the autograd graph.
"""
from __future__ import annotations

import torch

from ._binding import FmmError


class _PoissonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, plan, tol, restart, maxit):
        u = torch.zeros_like(f)
        info = plan.solve(f.contiguous(), u, tol=tol, restart=restart, maxit=maxit)
        if not info["converged"]:
            raise FmmError(1, "forward solve did not converge: %r" % (info,))
        ctx.plan, ctx.prm = plan, (tol, restart, maxit)
        ctx.info = info
        return u

    @staticmethod
    def backward(ctx, gu):
        tol, restart, maxit = ctx.prm
        lam = torch.zeros_like(gu)
        info = ctx.plan.solve_adjoint(gu.contiguous(), lam, tol=tol, restart=restart, maxit=maxit)
        if not info["converged"]:
            raise FmmError(1, "adjoint solve did not converge: %r" % (info,))
        return lam, None, None, None, None


class _GaussianBumps(torch.autograd.Function):
    @staticmethod
    def forward(ctx, cx, cy, w, a, plan):
        f = torch.empty(plan.npts, dtype=torch.float64, device=cx.device)
        plan.bumps_eval(cx.contiguous(), cy.contiguous(), w.contiguous(), a.contiguous(), f)
        ctx.save_for_backward(cx, cy, w, a)
        ctx.plan = plan
        return f

    @staticmethod
    def backward(ctx, gf):
        cx, cy, w, a = ctx.saved_tensors
        K = cx.numel()
        outs = [torch.empty(K, dtype=torch.float64, device=cx.device) if need else None
                for need in ctx.needs_input_grad[:4]]
        ctx.plan.bumps_grad(cx.contiguous(), cy.contiguous(), w.contiguous(), a.contiguous(),
                            gf.contiguous(), *outs)
        return outs[0], outs[1], outs[2], outs[3], None


def poisson_solve(plan, f, tol=1e-8, restart=30, maxit=600):
    """u = A^{-1} f (zero Dirichlet data), differentiable in f."""
    return _PoissonSolve.apply(f, plan, tol, restart, maxit)


def gaussian_bumps(plan, cx, cy, w, a):
    """f = sum_k a_k exp(-|x - c_k|^2 / (2 w_k^2)) on the plan's grid,
    differentiable in all four parameter vectors."""
    return _GaussianBumps.apply(cx, cy, w, a, plan)
