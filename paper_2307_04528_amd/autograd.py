"""Differentiable shell solve: u = H(alpha)^{-1} rhs as a torch.autograd.Function.

Backward (implicit function theorem): with L a scalar loss and w = dL/du,
    lambda = H^{-T} w            (adjoint solve, transposed V-cycle)
    dL/drhs = lambda,   dL/dalpha = -lambda * V * u
since dH/dalpha at a cell is the cell volume V on that cell's diagonal.
Both the solve and the adjoint run in the HIP library (mg_solve,
mg_solve_adjoint, mg_grad_alpha).
"""
from __future__ import annotations

import torch

from .solver import Solver


class MGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rhs: torch.Tensor, alpha: torch.Tensor, solver: Solver,
                tol: float = 1e-8):
        a = alpha.detach().contiguous()
        if not solver.alpha_is_current(a):
            solver.update_alpha(a)
        u, _ = solver.solve(rhs.detach().contiguous(), tol)
        ctx.solver = solver
        ctx.tol = tol
        # saved, so that an in-place change of alpha before backward raises
        ctx.save_for_backward(u, alpha)
        return u

    @staticmethod
    def backward(ctx, grad_u: torch.Tensor):
        u, alpha = ctx.saved_tensors
        solver: Solver = ctx.solver
        a = alpha.detach().contiguous()
        if not solver.alpha_is_current(a):
            # the solver has served another alpha since the forward solve
            solver.update_alpha(a)
        lam, _ = solver.solve_adjoint(grad_u.contiguous(), ctx.tol)
        g_alpha = solver.grad_alpha(lam, u) if ctx.needs_input_grad[1] else None
        g_rhs = lam if ctx.needs_input_grad[0] else None
        return g_rhs, g_alpha, None, None


def mg_solve(rhs: torch.Tensor, alpha: torch.Tensor, solver: Solver, tol: float = 1e-8):
    """u = H(alpha)^{-1} rhs, differentiable in rhs and alpha."""
    return MGSolve.apply(rhs, alpha, solver, tol)
