"""The single-workgroup Gl-BiCG / eGl-BiCG / Gl-BiCGStab path for small systems (n <= 1024,
s <= 4 real or s <= 2 complex, CSR, no preconditioner), through the C ABI:
against the oracle at a fixed iteration count and at convergence, and against
the general multi-kernel schedule (fused_small=False) on the same inputs."""
import sys

import numpy as np
import pytest

import inputs as I
import oracle as O

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def pkg():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1504_04395_amd as P
    P.load_library()
    return P


@pytest.fixture(scope="module")
def ctx(pkg):
    c = pkg.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def _matrix(kind, n):
    """Real: the 2D convection-diffusion operator (n = m^2) or the real part of a
    power-law matrix (ragged rows of 4..n-1 entries); complex: the power-law
    matrix.  Both power-law variants are strictly diagonally dominant."""
    if kind == "convdiff":
        m = int(round(np.sqrt(n)))
        assert m * m == n
        return I.convdiff2d(m)
    C = I.powerlaw(n=n, seed=n, lo=4, hi=min(400, n - 1), mean=min(20.0, (n - 1) / 2))
    if kind == "powerlaw_real":
        return I.CSR(C.n, C.indptr, C.indices, np.ascontiguousarray(C.data.real))
    return C


SHAPES = [("convdiff", 1024, s) for s in (1, 2, 3, 4)] + \
         [("convdiff", 49, 3), ("powerlaw_real", 1000, 4), ("powerlaw_real", 333, 2),
          ("powerlaw", 1000, 1), ("powerlaw", 1000, 2), ("powerlaw", 517, 2)]


FUSED = ["gl_bicg", "egl_bicg", "gl_bicgstab"]


@pytest.mark.parametrize("method", FUSED)
@pytest.mark.parametrize("kind,n,s", SHAPES)
def test_fixed_iterations_match_oracle(pkg, ctx, kind, n, s, method):
    """Eight iterations on both sides: iterates and history agree to 1e-10."""
    C = _matrix(kind, n)
    B = I.gaussian_block(C.n, s, seed=7 + s, complex_=C.is_complex)
    say("fused fixed", kind, n, s, method)
    ref = O.solve(C, B, method, tol=0.0, maxit=8)
    A = pkg.Matrix.from_csr(ctx, C)
    X, info = pkg.solve(ctx, A, B, method, tol=0.0, maxit=8)
    A.close()
    assert info.single_workgroup   # the single-workgroup kernel ran
    assert info.iterations == 8 and info.status == ref.status   # not converged, or diverged (||R_8|| > ||R_0||)
    assert info.matvecs == ref.matvecs
    assert _rel(X, ref.X) < 1e-10, _rel(X, ref.X)
    np.testing.assert_allclose(info.history, ref.history, rtol=1e-10, atol=0)


@pytest.mark.parametrize("method", FUSED)
@pytest.mark.parametrize("kind,n,s", SHAPES)
def test_converged_matches_general_schedule(pkg, ctx, kind, n, s, method):
    """To 1e-12: the fused path and the general schedule reach the same status,
    iteration counts within 2% (+1), X within 1e-10 of each other and of the
    oracle, and the true residual at the stopping level."""
    C = _matrix(kind, n)
    B = I.gaussian_block(C.n, s, seed=11 + s, complex_=C.is_complex)
    say("fused converged", kind, n, s, method)
    ref = O.solve(C, B, method, tol=1e-12, maxit=5000)
    A = pkg.Matrix.from_csr(ctx, C)
    X1, i1 = pkg.solve(ctx, A, B, method, tol=1e-12, maxit=5000)
    X2, i2 = pkg.solve(ctx, A, B, method, tol=1e-12, maxit=5000, fused_small=False)
    A.close()
    say(f"  fused it={i1.iterations} general it={i2.iterations} oracle it={ref.iterations} "
        f"res={i1.rel_res_true:.2e}")
    assert i1.single_workgroup and not i2.single_workgroup
    assert i1.status == i2.status == ref.status == 0
    assert abs(i1.iterations - i2.iterations) <= 1 + int(0.02 * i2.iterations)
    assert abs(i1.iterations - ref.iterations) <= 1 + int(0.05 * ref.iterations)
    m = min(8, len(i1.history), len(i2.history))
    np.testing.assert_allclose(i1.history[:m], i2.history[:m], rtol=1e-10, atol=0)
    assert _rel(X1, X2) < 1e-10 and _rel(X1, ref.X) < 1e-10
    assert i1.rel_res_true < 1e-11


@pytest.mark.parametrize("method", FUSED)
def test_one_row_and_size_limits(pkg, ctx, method):
    """n = 1 (without the QR preprocessing, which needs s <= n columns of full
    rank and reports a breakdown before the first iteration otherwise): one
    BiCG iteration solves it; BiCGStab's half step solves it too, and the zero
    T = A S then breaks the omega quotient, as in the oracle.  And n = 1024 /
    1025 on either side of the single-workgroup limit (the larger one runs the
    general schedule)."""
    C1 = I.CSR(1, np.array([0, 1], dtype=np.int64), np.array([0], dtype=np.int32), np.array([4.0]))
    B1 = np.array([[2.0, -1.0, 0.5, 3.0]])
    A = pkg.Matrix.from_csr(ctx, C1)
    X, info = pkg.solve(ctx, A, B1, method, tol=1e-12, preprocess_qr=False)
    ref = O.solve(C1, B1, method, tol=1e-12, preprocess=False)
    assert info.status == ref.status and info.iterations == ref.iterations
    if method == "gl_bicgstab":
        assert info.status_name == "breakdown" and info.breakdown_iter == 0 and np.all(X == 0)
    else:
        assert info.status_name == "ok" and info.iterations == 1
        np.testing.assert_allclose(X, B1 / 4.0, rtol=1e-15)
    X, info = pkg.solve(ctx, A, B1, method, tol=1e-12)
    assert info.status_name == "breakdown" and info.iterations == 0
    A.close()
    for n in (1024, 1025):
        C = I.powerlaw(n=n, seed=3, lo=4, hi=400, mean=20.0)
        C = I.CSR(C.n, C.indptr, C.indices, np.ascontiguousarray(C.data.real))
        B = I.gaussian_block(n, 3, seed=5)
        ref = O.solve(C, B, method, tol=0.0, maxit=6)
        A = pkg.Matrix.from_csr(ctx, C)
        X, info = pkg.solve(ctx, A, B, method, tol=0.0, maxit=6)
        A.close()
        assert info.single_workgroup == (n <= 1024)
        assert info.iterations == 6 and _rel(X, ref.X) < 1e-10


def test_zero_iterations_and_zero_rhs(pkg, ctx):
    """maxit = 0 stops before the first iteration (not converged, X = X0); a
    zero right-hand side without the QR preprocessing converges at once."""
    C = I.convdiff2d(16)
    B = I.gaussian_block(C.n, 2, seed=3)
    A = pkg.Matrix.from_csr(ctx, C)
    for method in FUSED:
        X, info = pkg.solve(ctx, A, B, method, maxit=0)
        assert info.status_name == "not_converged" and info.iterations == 0 and np.all(X == 0)
        X, info = pkg.solve(ctx, A, np.zeros_like(B), method, preprocess_qr=False)
        assert info.status_name == "ok" and info.iterations == 0 and np.all(X == 0)
    A.close()


def test_warm_start_and_adjoint(pkg, ctx):
    """X0 != 0 and the adjoint system A^H X = B also take the fused path and
    match the oracle after a fixed number of iterations."""
    C = I.powerlaw(n=800, seed=9, lo=4, hi=400, mean=20.0)
    B = I.gaussian_block(C.n, 2, seed=4, complex_=True)
    X0 = I.gaussian_block(C.n, 2, seed=5, complex_=True)
    A = pkg.Matrix.from_csr(ctx, C)
    for method in FUSED:
        ref = O.solve(C, B, method, X0=X0, tol=0.0, maxit=7)
        X, info = pkg.solve(ctx, A, B, method, X=X0.copy(), tol=0.0, maxit=7)
        assert info.iterations == 7 and _rel(X, ref.X) < 1e-10
        Sh = C.to_scipy().conj().T.tocsr()
        Sh.sort_indices()
        CH = I.CSR(C.n, Sh.indptr.astype(np.int64), Sh.indices.astype(np.int32), Sh.data)
        ref = O.solve(CH, B, method, tol=0.0, maxit=7)
        X, info = pkg.solve(ctx, A, B, method, tol=0.0, maxit=7, adjoint=True)
        assert info.iterations == 7 and _rel(X, ref.X) < 1e-10
    A.close()


def test_repeatable_bit_for_bit(pkg, ctx):
    """Every sum has a fixed order (no atomics, one workgroup): the same solve
    twice gives the same bits and the same iteration count."""
    C = I.convdiff2d(32)
    B = I.gaussian_block(C.n, 4, seed=2)
    A = pkg.Matrix.from_csr(ctx, C)
    for method in FUSED:
        X1, i1 = pkg.solve(ctx, A, B, method, tol=1e-10)
        X2, i2 = pkg.solve(ctx, A, B, method, tol=1e-10)
        assert i1.iterations == i2.iterations and np.array_equal(X1, X2)
        np.testing.assert_array_equal(i1.history, i2.history)
    A.close()


def test_history_copy_paths(pkg, ctx):
    """The residual history reaches the caller whole on both of its routes (a
    pinned copy enqueued behind the kernel for maxit + 1 <= 65536 entries, a
    blocking copy above that) and is cut to the caller's history_cap."""
    C = I.convdiff2d(32)
    B = I.gaussian_block(C.n, 4, seed=6)
    A = pkg.Matrix.from_csr(ctx, C)
    for method in FUSED:
        X1, i1 = pkg.solve(ctx, A, B, method, tol=1e-10, maxit=10000)
        X2, i2 = pkg.solve(ctx, A, B, method, tol=1e-10, maxit=100000)
        X3, i3 = pkg.solve(ctx, A, B, method, tol=1e-10, maxit=10000, history_cap=5)
        assert i1.single_workgroup and i2.single_workgroup and i3.single_workgroup
        assert i1.status_name == i2.status_name == "ok" and i1.iterations == i2.iterations == i3.iterations
        assert len(i1.history) == len(i2.history) == i1.iterations + 1
        np.testing.assert_array_equal(i1.history, i2.history)
        np.testing.assert_array_equal(i3.history, i1.history[:5])
        assert np.array_equal(X1, X2) and np.array_equal(X1, X3)
    A.close()


@pytest.mark.parametrize("method", FUSED)
def test_ill_conditioned_rhs_shifted_qr(pkg, ctx, method):
    """B with kappa about 1e9 (its third column the first plus 1e-9 noise): the
    plain Cholesky factorisation of B^H B fails its pivot test, so the
    preprocessing takes the shifted CholeskyQR2 (three passes).  The one-launch
    QR of the single-workgroup path and the general schedule's multi-kernel
    one then give the same converged X (1e-10), as does the oracle (its
    Householder QR), with the true residual at the stopping level."""
    C = I.convdiff2d(32)
    B = I.gaussian_block(C.n, 3, seed=21)
    noise = I.gaussian_block(C.n, 1, seed=22)[:, 0]
    B[:, 2] = B[:, 0] + 1e-9 * noise
    assert np.linalg.cond(B) > 1e8
    say("fused shifted QR", method)
    ref = O.solve(C, B, method, tol=1e-12, maxit=5000)
    A = pkg.Matrix.from_csr(ctx, C)
    X1, i1 = pkg.solve(ctx, A, B, method, tol=1e-12, maxit=5000)
    X2, i2 = pkg.solve(ctx, A, B, method, tol=1e-12, maxit=5000, fused_small=False)
    A.close()
    say(f"  fused it={i1.iterations} general it={i2.iterations} oracle it={ref.iterations} "
        f"res={i1.rel_res_true:.2e} {i2.rel_res_true:.2e}")
    assert i1.single_workgroup and not i2.single_workgroup
    assert i1.status_name == i2.status_name == "ok" and ref.status == 0
    assert abs(i1.iterations - i2.iterations) <= 1 + int(0.02 * i2.iterations)
    assert _rel(X1, X2) < 1e-10 and _rel(X1, ref.X) < 1e-10
    assert i1.rel_res_true < 1e-11 and i2.rel_res_true < 1e-11
