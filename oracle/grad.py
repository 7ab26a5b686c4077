"""Oracle for the differentiable solve X = A^{-1} B.

TEST INFRASTRUCTURE ONLY (see the package docstring).

For a real loss L(X) with G_X = dL/dX, the adjoint of X = A^{-1} B gives
    G_B = A^{-H} G_X,      dL/dA = -G_B X^H,
and the gradient with respect to the stored values of a sparse A is the
restriction of -G_B X^H to A's sparsity pattern (sampled dense-dense product).
"""
from __future__ import annotations

import numpy as np


def sddmm(indptr, indices, G, X, scale=-1.0):
    """out[k] = scale * sum_c G[i_k, c] * conj(X[j_k, c]) for every stored entry
    k = (i_k, j_k) of the pattern (row pointers ``indptr``, columns ``indices``)."""
    n = len(indptr) - 1
    rows = np.repeat(np.arange(n), np.diff(indptr))
    return scale * np.einsum("kc,kc->k", G[rows], np.conj(X[indices]))


def dense_solve_grad(A_dense, B, G_X):
    """Dense LU reference: X = A^{-1} B, G_B = A^{-H} G_X, G_A = -G_B X^H (dense)."""
    X = np.linalg.solve(A_dense, B)
    G_B = np.linalg.solve(A_dense.conj().T, G_X)
    G_A = -G_B @ X.conj().T
    return X, G_B, G_A
