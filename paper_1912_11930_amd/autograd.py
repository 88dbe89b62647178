"""Differentiable solve X = A(values)^{-1} B and stencil assembly values(kappa).

Backward of the solve (A symmetric): Y = A^{-1} G by a second block CG solve
with the same matrix gives dL/dB = Y, and dL/dvalues[e] = -<Y[row e], X[col e]>
(the dense -Y X^T sampled on A's pattern, one HIP kernel). Backward of the
assembly is the transpose Jacobian of the face-coefficient formula (one HIP
kernel).
"""
from __future__ import annotations

import torch

from .solver import BCG, stencil, stencil_kappa_vjp


class BCGSolve(torch.autograd.Function):
    """X = BCGSolve.apply(values, B, solver, tol, maxit)."""

    @staticmethod
    def forward(ctx, values: torch.Tensor, B: torch.Tensor, solver: BCG, tol: float = 1e-10, maxit: int = 100000):
        values = values.detach().contiguous()
        solver.update_values(values)
        X, info = solver.solve(B.detach().contiguous(), tol=tol, maxit=maxit)
        if info["status"] < 0:
            raise RuntimeError(f"forward solve failed: {info['status_name']}")
        ctx.solver, ctx.tol, ctx.maxit = solver, tol, maxit
        ctx.info = info
        ctx.save_for_backward(values, X)
        return X

    @staticmethod
    def backward(ctx, G: torch.Tensor):
        values, X = ctx.saved_tensors
        solver: BCG = ctx.solver
        solver.update_values(values)      # the adjoint uses the forward's A
        Y, info = solver.solve(G.contiguous(), tol=ctx.tol, maxit=ctx.maxit)
        if info["status"] < 0:
            raise RuntimeError(f"adjoint solve failed: {info['status_name']}")
        dvals = solver.csr_outer(Y, X, -1.0) if ctx.needs_input_grad[0] else None
        dB = Y if ctx.needs_input_grad[1] else None
        return dvals, dB, None, None, None


class StencilValues(torch.autograd.Function):
    """values = StencilValues.apply(kappa, dim, N) on the fixed stencil pattern."""

    @staticmethod
    def forward(ctx, kappa: torch.Tensor, dim: int, N: int):
        kappa = kappa.detach().contiguous()
        _, _, values = stencil(dim, N, kappa)
        ctx.save_for_backward(kappa)
        ctx.dim, ctx.N = dim, N
        return values

    @staticmethod
    def backward(ctx, dvalues: torch.Tensor):
        (kappa,) = ctx.saved_tensors
        return stencil_kappa_vjp(ctx.dim, ctx.N, kappa, dvalues.contiguous()), None, None
