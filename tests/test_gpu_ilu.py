"""GPU parity for right no-fill ILU preconditioning (Section 5.2): the
level-scheduled triangular solves against the oracle's, and preconditioned
solves of several methods against the oracle's preconditioned solves, on the
same seeded inputs, through the C ABI."""
import sys

import numpy as np
import pytest

import inputs as I
import oracle as O
from oracle.ilu import RightILU

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


def _problem(name):
    if name.startswith("ex"):
        P = I.paper_example(int(name[2]), "small")
        return P.A, P.B
    P = I.config(int(name[3]), "small")
    if name == "cfg3":
        return P.A, I.gaussian_block(P.A.n, 12, seed=0, complex_=True)
    return P.A, P.B


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3", "cfg4", "ex1", "ex2"])
@pytest.mark.parametrize("s", [1, 5, 16, 19, 32])
@pytest.mark.parametrize("adjoint", [False, True])
def test_precond_apply_matches_oracle(pkg, ctx, name, s, adjoint):
    A_, _ = _problem(name)
    cplx = np.iscomplexobj(A_.data)
    Z = I.gaussian_block(A_.n, s, seed=11, complex_=cplx)
    M = RightILU(A_.to_scipy().tocsr())
    ref = M.minv_h(Z) if adjoint else M.minv(Z)
    if ref.ndim == 1:
        ref = ref.reshape(-1, 1)
    A = pkg.Matrix.from_csr(ctx, A_).ilu0()
    Y = pkg.precond_apply(ctx, A, Z, adjoint=adjoint)
    A.close()
    err = _rel(Y, ref)
    say(f"{name} s={s} adjoint={adjoint}: rel err {err:.2e}")
    assert err < 1e-12


def test_precond_apply_device_in_place(pkg, ctx):
    import torch
    A_, _ = _problem("ex2")
    Z = I.gaussian_block(A_.n, 19, seed=3)
    ref = RightILU(A_.to_scipy().tocsr()).minv(Z)
    A = pkg.Matrix.from_csr(ctx, A_).ilu0()
    Zd = torch.from_numpy(Z).cuda()
    pkg.precond_apply(ctx, A, Zd, Y=Zd)
    torch.cuda.synchronize()
    A.close()
    assert _rel(Zd.cpu().numpy(), ref) < 1e-12


def _spread(A_, B, method, ref, seeds, **kw):
    xs, its, runs = 0.0, 0, []
    for sd in seeds:
        rng = np.random.default_rng(sd)
        noise = rng.standard_normal(B.shape)
        if np.iscomplexobj(B):
            noise = noise + 1j * rng.standard_normal(B.shape)
        r2 = O.solve(A_, B * (1 + 1e-15 * noise), method, precond="ilu0", **kw)
        xs = max(xs, _rel(r2.X, ref.X))
        its = max(its, abs(r2.iterations - ref.iterations))
        runs.append(r2)
    return xs, its, runs


CASES = [("ex1", m) for m in ("bl_bicg_rq", "bl_bicgstab_rq", "bl_bicgstab", "egl_qmr", "gl_bicgstab")] + \
        [("ex2", m) for m in ("bl_bicg_rq", "bl_bicgstab_rq", "egl_bicg", "gl_qmr", "li_qmr")] + \
        [("ex3", m) for m in ("bl_bicg", "bl_bicgstab", "li_bicg", "li_bicgstab")] + \
        [("cfg3", m) for m in ("bl_bicg_rq", "egl_qmr", "gl_bicg")] + \
        [("cfg4", m) for m in ("bl_bicgstab_rq", "egl_bicg")]


@pytest.mark.parametrize("name,method", CASES)
def test_fixed_iterations_match_oracle(pkg, ctx, name, method):
    """Five preconditioned iterations: X = M^-1 D R_R and the residual history
    agree with the oracle to 1e-10 (or 100x its own spread)."""
    A_, B = _problem(name)
    it = 5
    ref = O.solve(A_, B, method, tol=0.0, maxit=it, precond="ilu0")
    xs, _, _ = _spread(A_, B, method, ref, (12345,), tol=0.0, maxit=it)
    A = pkg.Matrix.from_csr(ctx, A_).ilu0()
    X, info = pkg.solve(ctx, A, B, method, tol=0.0, maxit=it, precond="ilu0")
    A.close()
    say(f"{name} {method}: gpu it={info.iterations} st={info.status_name} | oracle it={ref.iterations} "
        f"st={ref.status} | err={_rel(X, ref.X):.2e} spread={xs:.2e}")
    assert info.status == ref.status and info.iterations == ref.iterations
    if ref.status == O.STATUS_BREAKDOWN:
        return
    assert _rel(X, ref.X) < max(1e-10, 100 * xs)
    np.testing.assert_allclose(info.history, ref.history, rtol=1e-9, atol=0)
    assert info.matvecs == ref.matvecs


@pytest.mark.parametrize("name,method", CASES)
def test_solve_matches_oracle(pkg, ctx, name, method):
    """To tol 1e-10 (at most 300 iterations), as in Section 5.2: where the oracle
    and three 1e-15 perturbations of B all converge, the GPU converges within 5%
    of the iterations plus that spread, to the same X; otherwise it ends in one
    of the oracle's outcomes."""
    A_, B = _problem(name)
    tol, maxit = 1e-10, 300
    ref = O.solve(A_, B, method, tol=tol, maxit=maxit, precond="ilu0")
    xs, its, runs = _spread(A_, B, method, ref, (12345, 7, 99), tol=tol, maxit=maxit)
    A = pkg.Matrix.from_csr(ctx, A_).ilu0()
    X, info = pkg.solve(ctx, A, B, method, tol=tol, maxit=maxit, precond="ilu0")
    A.close()
    say(f"{name} {method}: gpu st={info.status_name} it={info.iterations} res={info.rel_res_true:.1e} | "
        f"oracle st={ref.status} it={ref.iterations} res={ref.rel_res_true:.1e} | perturbed "
        f"st={[r.status for r in runs]} it={[r.iterations for r in runs]} | err={_rel(X, ref.X):.1e} spread={xs:.1e}")
    m = min(6, len(ref.history), len(info.history))
    np.testing.assert_allclose(info.history[:m], ref.history[:m], rtol=1e-9, atol=0)
    outcomes = {ref.status} | {r.status for r in runs}
    if outcomes == {O.STATUS_OK} and xs < 1e-6:
        assert info.status == 0
        assert abs(info.iterations - ref.iterations) <= max(1, int(0.05 * ref.iterations)) + its
        assert _rel(X, ref.X) <= max(1e-9, 100 * xs)
        assert info.rel_res_true < 2e-10
    else:
        assert info.status in outcomes, (info.status, outcomes)


def test_ilu_requirements(pkg, ctx):
    """precond='ilu0' needs the factors; new values drop them; FP32 refinement
    and adjoint solves reject preconditioning."""
    A_, B = _problem("ex1")
    A = pkg.Matrix.from_csr(ctx, A_)
    with pytest.raises(pkg.SkrError):
        pkg.solve(ctx, A, B, "gl_bicg", precond="ilu0")
    A.ilu0()
    _, info = pkg.solve(ctx, A, B, "gl_bicg", tol=1e-8, precond="ilu0")
    assert info.status == 0
    with pytest.raises(pkg.SkrError):
        pkg.solve(ctx, A, B, "gl_bicg", precond="ilu0", precision="fp32_refine")
    with pytest.raises(pkg.SkrError):
        pkg.solve(ctx, A, B, "gl_bicg", precond="ilu0", adjoint=True)
    A.update_values(A_.data * 1.0)
    with pytest.raises(pkg.SkrError):
        pkg.solve(ctx, A, B, "gl_bicg", precond="ilu0")
    A.close()


def test_ilu_rejects_missing_diagonal(pkg, ctx):
    n = 4
    indptr = np.array([0, 1, 3, 5, 7], dtype=np.int64)
    indices = np.array([1, 0, 1, 1, 2, 2, 3], dtype=np.int32)   # row 0 has no diagonal
    data = np.ones(7)
    A = pkg.Matrix(ctx, n, indptr, indices, data)
    with pytest.raises(pkg.SkrError):
        A.ilu0()
    A.close()


def test_ilu_with_sell_storage_warm_start_and_no_preprocessing(pkg, ctx):
    """ILU(0) with SELL-C-sigma storage of A (the factors come from the CSR
    values either way), with a nonzero initial guess, and without the QR
    preprocessing of R0: each against the oracle's preconditioned solve."""
    A_, B = _problem("cfg4")
    method = "bl_bicgstab_rq"
    ref = O.solve(A_, B, method, tol=1e-10, maxit=200, precond="ilu0")
    for fmt in ("csr", "sell"):
        A = pkg.Matrix.from_csr(ctx, A_, fmt=fmt).ilu0()
        X, info = pkg.solve(ctx, A, B, method, tol=1e-10, maxit=200, precond="ilu0")
        A.close()
        say(f"{fmt}: it={info.iterations} (oracle {ref.iterations}) err={_rel(X, ref.X):.1e}")
        assert info.status == 0 and abs(info.iterations - ref.iterations) <= 1
        assert _rel(X, ref.X) < 1e-8
    X0 = 0.5 * I.gaussian_block(A_.n, B.shape[1], seed=21, complex_=True)
    for pre in (True, False):
        ref = O.solve(A_, B, "egl_bicg", tol=1e-10, maxit=200, precond="ilu0", X0=X0, preprocess=pre)
        A = pkg.Matrix.from_csr(ctx, A_).ilu0()
        X, info = pkg.solve(ctx, A, B, "egl_bicg", X=X0.copy(), tol=1e-10, maxit=200, precond="ilu0",
                            preprocess_qr=pre)
        A.close()
        say(f"warm start, preprocess={pre}: it={info.iterations} (oracle {ref.iterations}) "
            f"err={_rel(X, ref.X):.1e}")
        assert info.status == 0 and abs(info.iterations - ref.iterations) <= 1
        assert _rel(X, ref.X) < 1e-8
        np.testing.assert_allclose(info.history[:5], ref.history[:5], rtol=1e-9, atol=0)
