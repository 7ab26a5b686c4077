"""No-fill incomplete LU factorisation and right preconditioning (Section 5.2:
Examples 1-3 are also solved with a right ILU preconditioner without fill).

TEST INFRASTRUCTURE ONLY (see the package docstring).

ILU(0) (Saad, Iterative Methods for Sparse Linear Systems, Section 10.3.2):
A = L U - E with L unit lower triangular and U upper triangular, both on A's
sparsity pattern, and (L U)_ij = a_ij for every (i, j) in the pattern.  The
factors come from Gaussian elimination in row order that drops every update
falling outside the pattern:

    for i = 1..n-1, for k < i with (i, k) in the pattern, in increasing k:
        a_ik <- a_ik / a_kk
        a_ij <- a_ij - a_ik a_kj   for j > k with (i, j) and (k, j) in the pattern

Right preconditioning with M = L U solves (A M^-1) Y = B and returns
X = M^-1 Y; the residual B - A M^-1 Y is that of X, so stopping rules and
residual histories keep their meaning.  The products the methods need are
A M^-1 Z = A (U^-1 (L^-1 Z)) and (A M^-1)^H Z = M^-H (A^H Z) =
L^-H (U^-H (A^H Z)).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular


class ZeroPivot(ValueError):
    pass


def _csr32(M):
    """CSR with C-int index arrays (what scipy's triangular solver takes)."""
    M = sp.csr_array(M)
    M.sort_indices()
    M.indices = M.indices.astype(np.intc)
    M.indptr = M.indptr.astype(np.intc)
    return M


def ilu0(A):
    """ILU(0) of a square sparse matrix with a full diagonal: returns (L, U) as
    CSR matrices, L unit lower triangular (diagonal stored), U upper triangular."""
    A = sp.csr_array(A)
    A.sort_indices()
    n = A.shape[0]
    rows = []
    for i in range(n):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        rows.append(dict(zip(A.indices[lo:hi].tolist(), A.data[lo:hi].tolist())))
    for i in range(n):
        ri = rows[i]
        if i not in ri:
            raise ZeroPivot(f"row {i} has no diagonal entry")
        for k in sorted(c for c in ri if c < i):
            ukk = rows[k][k]
            if ukk == 0:
                raise ZeroPivot(f"zero pivot in row {k}")
            lik = ri[k] / ukk
            ri[k] = lik
            for j, ukj in rows[k].items():
                if j > k and j in ri:
                    ri[j] = ri[j] - lik * ukj
        if ri[i] == 0:
            raise ZeroPivot(f"zero pivot in row {i}")
    Li, Lj, Lv, Ui, Uj, Uv = [], [], [], [], [], []
    for i, ri in enumerate(rows):
        for j, v in ri.items():
            if j < i:
                Li.append(i), Lj.append(j), Lv.append(v)
            else:
                Ui.append(i), Uj.append(j), Uv.append(v)
        Li.append(i), Lj.append(i), Lv.append(1.0)
    dt = A.dtype
    L = sp.csr_array((np.array(Lv, dtype=dt), (Li, Lj)), shape=(n, n))
    U = sp.csr_array((np.array(Uv, dtype=dt), (Ui, Uj)), shape=(n, n))
    return _csr32(L), _csr32(U)


class RightILU:
    """M = L U from ilu0(A); applies M^-1 and M^-H to blocks."""

    def __init__(self, A):
        self.L, self.U = ilu0(A)
        self.LH = _csr32(self.L.conj().T)
        self.UH = _csr32(self.U.conj().T)

    def minv(self, Z):
        Y = spsolve_triangular(self.L, Z, lower=True, unit_diagonal=True)
        return spsolve_triangular(self.U, Y, lower=False)

    def minv_h(self, Z):
        Y = spsolve_triangular(self.UH, Z, lower=True)
        return spsolve_triangular(self.LH, Y, lower=False, unit_diagonal=True)


class PrecOp:
    """The right-preconditioned operator A M^-1 (``adjoint=False``) or its
    adjoint M^-H A^H (``adjoint=True``), applied with ``@`` to n x s blocks."""

    def __init__(self, A, AH, M: RightILU, adjoint: bool):
        self.A, self.AH, self.M, self.adjoint = A, AH, M, adjoint

    def __matmul__(self, Z):
        if self.adjoint:
            return self.M.minv_h(self.AH @ Z)
        return self.A @ self.M.minv(Z)
