"""Pins for the oracle's no-fill ILU and right preconditioning (Section 5.2)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import inputs as I
import oracle as O
from oracle.ilu import RightILU, ZeroPivot, ilu0


def _real(m=12):
    return I.convdiff2d(m, (20.0, 20.0)).to_scipy().tocsr()


def _complex(n=300):
    return I.powerlaw(n, seed=7, lo=4, hi=20, mean=8.0).to_scipy().tocsr()


def _tridiag(n=40, cplx=False, seed=3):
    rng = np.random.default_rng(seed)
    lo, up = rng.standard_normal(n - 1), rng.standard_normal(n - 1)
    d = 4.0 + rng.random(n)
    if cplx:
        lo = lo + 1j * rng.standard_normal(n - 1)
        up = up + 1j * rng.standard_normal(n - 1)
    return sp.diags([lo, d, up], [-1, 0, 1], format="csr")


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_ilu0_defining_property(kind):
    """L unit lower and U upper on A's pattern, and L U = A on that pattern
    (this characterises ILU(0)); the fill that L U has off the pattern is
    dropped, so L U differs from A there."""
    A = _real() if kind == "real" else _complex()
    L, U = ilu0(A)
    Ad, Ld, Ud = A.toarray(), L.toarray(), U.toarray()
    pat = Ad != 0
    assert np.allclose(np.diag(Ld), 1.0)
    assert np.all(Ld[np.triu_indices_from(Ld, 1)] == 0)
    assert np.all(Ud[np.tril_indices_from(Ud, -1)] == 0)
    assert not np.any((np.tril(Ld, -1) != 0) & ~pat)
    assert not np.any((Ud != 0) & ~pat)
    LU = Ld @ Ud
    scale = np.abs(Ad).max()
    assert np.abs(LU[pat] - Ad[pat]).max() < 1e-13 * scale
    assert np.abs(LU[~pat]).max() > 1e-6 * scale


@pytest.mark.parametrize("cplx", [False, True])
def test_ilu0_is_exact_lu_without_fill(cplx):
    """A tridiagonal matrix has no fill: ILU(0) is its LU factorisation (here
    without pivoting, which the diagonal dominance makes the pivoted one too)."""
    A = _tridiag(cplx=cplx)
    L, U = ilu0(A)
    P, Lr, Ur = sla.lu(A.toarray())
    assert np.allclose(P, np.eye(A.shape[0]))
    assert _rel(L.toarray(), Lr) < 1e-14
    assert _rel(U.toarray(), Ur) < 1e-14


def test_ilu0_reports_zero_pivot():
    A = sp.csr_array(np.array([[0.0, 1.0], [1.0, 1.0]]))
    with pytest.raises(ZeroPivot):
        ilu0(A)


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_minv_and_its_adjoint(kind):
    """M^-1 inverts L U, and M^-H is its adjoint: <M^-1 x, y> = <x, M^-H y>."""
    A = _real() if kind == "real" else _complex()
    M = RightILU(A)
    n = A.shape[0]
    X = I.gaussian_block(n, 3, seed=1, complex_=kind == "complex")
    Y = I.gaussian_block(n, 3, seed=2, complex_=kind == "complex")
    Z = M.minv(X)
    assert _rel(M.L @ (M.U @ Z), X) < 1e-13
    lhs = np.vdot(Y, Z)
    rhs = np.vdot(M.minv_h(Y), X)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("method", list(O.METHODS) + list(O.PIN_METHODS))
@pytest.mark.parametrize("kind", ["real", "complex"])
def test_preconditioned_solutions_match_dense_lu(method, kind):
    if kind == "real":
        A = _real(16)
        B = I.gaussian_block(A.shape[0], 4, seed=1)
    else:
        A = _complex(400)
        B = I.gaussian_block(A.shape[0], 3, seed=1, complex_=True)
    r = O.solve(A, B, method, tol=1e-12, maxit=2000, precond="ilu0")
    assert r.status == O.STATUS_OK, (method, r.status, r.iterations)
    Xd = np.linalg.solve(A.toarray(), B)
    kappa = np.linalg.cond(A.toarray())
    assert _rel(r.X, Xd) <= 10 * kappa * 1e-12
    assert r.rel_res_true < 1e-10


@pytest.mark.parametrize("method", ["gl_bicg", "egl_bicg", "gl_qmr", "egl_qmr", "bl_bicg", "bl_bicg_rq",
                                    "li_bicg", "li_qmr"])
@pytest.mark.parametrize("cplx", [False, True])
def test_exact_preconditioner_converges_in_one_iteration(method, cplx):
    """With no fill, M = A and A M^-1 = I: the BiCG and QMR variants stop after
    one iteration with the exact solution.  (The BiCGStab variants are left out:
    their intermediate residual is exactly zero then, which is a breakdown of
    the step length by the rule used here.)"""
    A = _tridiag(cplx=cplx)
    B = I.gaussian_block(A.shape[0], 3, seed=4, complex_=cplx)
    r = O.solve(A, B, method, tol=1e-12, maxit=10, precond="ilu0")
    assert r.status == O.STATUS_OK and r.iterations == 1, (r.status, r.iterations)
    assert _rel(r.X, np.linalg.solve(A.toarray(), B)) < 1e-13
