"""Differentiable sparse solve X = A^{-1} B on the GPU.

Forward: the simultaneous Krylov solver (``skr_solve``) on A.  Backward: for a
loss L with G_X = dL/dX, the adjoint of X = A^{-1} B gives

    G_B = A^{-H} G_X        (the same solver on A^H: ``skr_solve`` with adjoint=1)
    dL/dA = -G_B X^H        restricted to A's stored pattern (``skr_sddmm``).

The value gradient is returned for A's stored values in CSR order.  This is
argument marshalling only: both solves and the sampled product run in the HIP
library.
"""
from __future__ import annotations

import torch

from . import _binding as B


class SparseSolve(torch.autograd.Function):
    """X = SparseSolve.apply(values, rhs, matrix, method, tol, precision, maxit).

    ``values``: A's stored values (CSR order, length nnz, float64 or
    complex128, on the GPU); ``rhs``: n x s tensor; ``matrix``: a
    :class:`paper_1504_04395_amd.Matrix` with A's pattern, whose values are
    replaced by ``values`` before the forward solve."""

    @staticmethod
    def forward(ctx, values, rhs, matrix, method="egl_bicg", tol=1e-10, precision="fp64", maxit=20000):
        vals = values.detach().contiguous()
        matrix.update_values(vals)
        X, info = B.solve(matrix.ctx, matrix, rhs.detach().contiguous(), method, tol=tol, maxit=maxit,
                          precision=precision)
        if info.status != 0:
            raise RuntimeError(f"forward solve did not converge: {info.status_name} after {info.iterations} it")
        ctx.matrix = matrix
        ctx.opts = (method, tol, precision, maxit)
        ctx.save_for_backward(X)
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, grad_x):
        (X,) = ctx.saved_tensors
        method, tol, precision, maxit = ctx.opts
        A = ctx.matrix
        G_B, info = B.solve(A.ctx, A, grad_x.contiguous(), method, tol=tol, maxit=maxit, precision=precision,
                            adjoint=True)
        if info.status != 0:
            raise RuntimeError(f"adjoint solve did not converge: {info.status_name} after {info.iterations} it")
        grad_vals = B.sddmm(A.ctx, A, G_B, X, scale=-1.0) if ctx.needs_input_grad[0] else None
        return grad_vals, (G_B if ctx.needs_input_grad[1] else None), None, None, None, None, None


def sparse_solve(values, rhs, matrix, method="egl_bicg", tol=1e-10, precision="fp64", maxit=20000):
    """Functional form of :class:`SparseSolve`."""
    return SparseSolve.apply(values, rhs, matrix, method, tol, precision, maxit)
