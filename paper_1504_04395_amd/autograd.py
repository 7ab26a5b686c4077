"""Differentiable sparse solve X = A^{-1} B on the GPU.

Forward: the simultaneous Krylov solver (``skr_solve``) on A.  Backward: for a
loss L with G_X = dL/dX, the adjoint of X = A^{-1} B gives

    G_B = A^{-H} G_X        (the same solver on A^H: ``skr_solve`` with adjoint=1)
    dL/dA = -G_B X^H        restricted to A's stored pattern (``skr_sddmm``).

The value gradient is returned for A's stored values in CSR order.  This is
argument marshalling only: both solves and the sampled product run in the HIP
library.

Several solves may share one Matrix before a single backward pass.  Each
forward pass keeps the values it solved with and the matrix's version after
uploading them; a backward pass whose matrix has been updated since re-uploads
its own values first, so its adjoint solve and SDDMM see the A of its forward
pass.
"""
from __future__ import annotations

import torch

from . import _binding as B


class SparseSolve(torch.autograd.Function):
    """X = SparseSolve.apply(values, rhs, matrix, method, tol, precision, maxit, max_outer).

    ``values``: A's stored values (CSR order, length nnz, float64 or
    complex128, on the GPU); ``rhs``: n x s tensor; ``matrix``: a
    :class:`paper_1504_04395_amd.Matrix` with A's pattern, whose values are
    replaced by ``values`` before the forward solve."""

    @staticmethod
    def forward(ctx, values, rhs, matrix, method="egl_bicg", tol=1e-10, precision="fp64", maxit=20000,
                max_outer=30):
        vals = values.detach().contiguous()
        matrix.update_values(vals)
        X, info = B.solve(matrix.ctx, matrix, rhs.detach().contiguous(), method, tol=tol, maxit=maxit,
                          precision=precision, max_outer=max_outer)
        if info.status != 0:
            raise RuntimeError(f"forward solve did not converge: {info.status_name} after {info.iterations} it "
                               f"({info.outer_iterations} outer steps, true rel. residual {info.rel_res_true:.2e})")
        ctx.matrix = matrix
        ctx.version = matrix.version
        ctx.opts = (method, tol, precision, maxit, max_outer)
        ctx.save_for_backward(X, vals)
        ctx.info = info
        return X

    @staticmethod
    def backward(ctx, grad_x):
        X, vals = ctx.saved_tensors
        method, tol, precision, maxit, max_outer = ctx.opts
        A = ctx.matrix
        if A.version != ctx.version:   # another solve changed A's values since this forward pass
            A.update_values(vals)
        G_B, info = B.solve(A.ctx, A, grad_x.contiguous(), method, tol=tol, maxit=maxit, precision=precision,
                            max_outer=max_outer, adjoint=True)
        if info.status != 0:
            raise RuntimeError(f"adjoint solve did not converge: {info.status_name} after {info.iterations} it "
                               f"({info.outer_iterations} outer steps, true rel. residual {info.rel_res_true:.2e})")
        grad_vals = B.sddmm(A.ctx, A, G_B, X, scale=-1.0) if ctx.needs_input_grad[0] else None
        return grad_vals, (G_B if ctx.needs_input_grad[1] else None), None, None, None, None, None, None


def sparse_solve(values, rhs, matrix, method="egl_bicg", tol=1e-10, precision="fp64", maxit=20000, max_outer=30):
    """Functional form of :class:`SparseSolve`.  ``max_outer`` caps the outer
    FP64 refinement steps of ``precision='fp32_refine'`` (forward and adjoint
    solve alike)."""
    return SparseSolve.apply(values, rhs, matrix, method, tol, precision, maxit, max_outer)
