"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs."""
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

import inputs as I
import oracle as O

pytestmark = pytest.mark.gpu

METHODS = ["gl_bicg", "egl_bicg", "gl_qmr", "egl_qmr", "gl_bicgstab", "bl_bicg_rq", "bl_bicgstab_rq"]


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


# ---------------------------------------------------------------- SpMM
def _ragged_matrix(n, complex_, seed):
    """Random sparse matrix with empty rows, a few long rows and a ragged tail."""
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 9, size=n)
    lens[rng.choice(n, size=max(1, n // 50), replace=False)] = 0
    lens[rng.choice(n, size=3, replace=False)] = min(n, 300)
    rows, cols = [], []
    for i, L in enumerate(lens):
        c = np.sort(rng.choice(n, size=int(min(L, n)), replace=False))
        rows.append(np.full(len(c), i)); cols.append(c)
    rows = np.concatenate(rows); cols = np.concatenate(cols)
    vals = rng.standard_normal(rows.size)
    if complex_:
        vals = vals + 1j * rng.standard_normal(rows.size)
    M = sp.csr_array((vals, (rows, cols)), shape=(n, n))
    M.sort_indices()
    return I.CSR(n, M.indptr.astype(np.int64), M.indices.astype(np.int32), M.data)


@pytest.mark.parametrize("fmt", ["csr", "sell"])
@pytest.mark.parametrize("kind", ["real", "complex"])
@pytest.mark.parametrize("s", [1, 2, 3, 4, 8, 12, 16, 17, 32])
def test_spmm_matches_scipy(pkg, ctx, fmt, kind, s):
    n = 1000 + 37
    C = _ragged_matrix(n, kind == "complex", seed=s)
    say("spmm", fmt, kind, s)
    A = pkg.Matrix.from_csr(ctx, C, fmt=fmt, sell_C=32, sell_sigma=128)
    X = I.gaussian_block(n, s, seed=s + 1, complex_=(kind == "complex"))
    Sa = C.to_scipy()
    for adj in (False, True):
        Y = pkg.spmm(ctx, A, X, adjoint=adj)
        ref = (Sa.conj().T @ X) if adj else (Sa @ X)
        scale = np.abs(Sa).max() * np.abs(X).max() * 300
        np.testing.assert_allclose(Y, ref, rtol=0, atol=1e-14 * scale)
    A.close()


def _sell_slots(indptr, C, sigma):
    """Stored slots of SELL-C-sigma by its definition: rows sorted by length
    (longest first) inside windows of sigma rows, chunks of C consecutive sorted
    rows, each chunk padded to its longest row."""
    lens = np.diff(np.asarray(indptr))
    n = lens.size
    order = np.concatenate([w0 + np.argsort(-lens[w0:w0 + sigma], kind="stable") for w0 in range(0, n, sigma)])
    sl = lens[order]
    return sum(int(sl[c:c + C].max()) * C for c in range(0, n, C))


@pytest.mark.parametrize("C,sigma", [(16, 16), (16, 256), (64, 64), (64, 256)])
@pytest.mark.parametrize("kind,s", [("real", 4), ("real", 16), ("complex", 12), ("complex", 32)])
def test_sell_chunk_sizes(pkg, ctx, C, sigma, kind, s):
    """SELL-C-sigma with C = 16 and 64 (the other tests use C = 32): products with
    A and A^H against scipy, and the padding ratio against its definition."""
    n = 1000 + 37
    M = _ragged_matrix(n, kind == "complex", seed=C + s)
    say("sell", C, sigma, kind, s)
    A = pkg.Matrix.from_csr(ctx, M, fmt="sell", sell_C=C, sell_sigma=sigma)
    assert A.sell_padding == pytest.approx(_sell_slots(M.indptr, C, sigma) / M.nnz, rel=0, abs=1e-12)
    X = I.gaussian_block(n, s, seed=s + 7, complex_=(kind == "complex"))
    Sa = M.to_scipy()
    for adj in (False, True):
        Y = pkg.spmm(ctx, A, X, adjoint=adj)
        ref = (Sa.conj().T @ X) if adj else (Sa @ X)
        scale = np.abs(Sa).max() * np.abs(X).max() * 300
        np.testing.assert_allclose(Y, ref, rtol=0, atol=1e-14 * scale)
    A.close()


def test_spmm_device_tensors(pkg, ctx):
    import torch
    P = I.config(2, "small")
    A = pkg.Matrix.from_csr(ctx, P.A)
    Xd = torch.from_numpy(P.B).cuda()
    Y = pkg.spmm(ctx, A, Xd)
    torch.cuda.synchronize()
    np.testing.assert_allclose(Y.cpu().numpy(), P.A.to_scipy() @ P.B, rtol=1e-13, atol=1e-13)
    A.close()


# ---------------------------------------------------------------- QR and SDDMM
@pytest.mark.parametrize("kind", ["real", "complex"])
@pytest.mark.parametrize("s", [1, 4, 12, 16, 32])
def test_block_qr(pkg, ctx, kind, s):
    Z = I.gaussian_block(5000 + 3, s, seed=s, complex_=(kind == "complex"))
    Q, Cm, rc = pkg.block_qr(ctx, Z)
    assert rc == 0
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(s), atol=1e-13)
    np.testing.assert_allclose(Q @ Cm, Z, atol=1e-12 * np.abs(Z).max())
    Qo, Co = O.qr_pos(Z)            # unique QR with positive diagonal
    assert _rel(Cm, Co) < 1e-12
    assert np.allclose(np.tril(Cm, -1), 0)


@pytest.mark.parametrize("kind,s", [("real", 8), ("real", 24), ("complex", 8), ("complex", 32)])
def test_block_qr_ill_conditioned_uses_shift(pkg, ctx, kind, s):
    """kappa = 1e9: the shifted first pass plus two plain passes (three inverse
    factors applied in one final pass) on the real s <= 16 tiles and on the
    complex / wider tiles."""
    rng = np.random.default_rng(3)
    cplx = kind == "complex"

    def g(*shape):
        x = rng.standard_normal(shape)
        return x + 1j * rng.standard_normal(shape) if cplx else x

    U, _ = np.linalg.qr(g(4000, s))
    Z = U @ np.diag(np.logspace(0, -9, s)) @ np.linalg.qr(g(s, s))[0]
    assert np.linalg.cond(Z) > 1e8       # kappa^2 u > 1: the unshifted Cholesky of Z^H Z fails
    Q, Cm, rc = pkg.block_qr(ctx, Z)
    assert rc == 0
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(s), atol=1e-12)
    np.testing.assert_allclose(Q @ Cm, Z, atol=1e-13)


@pytest.mark.parametrize("kind", ["real", "complex"])
@pytest.mark.parametrize("s", [1, 3, 8, 32])
def test_sddmm(pkg, ctx, kind, s):
    n = 777
    C = _ragged_matrix(n, kind == "complex", seed=40 + s)
    A = pkg.Matrix.from_csr(ctx, C)
    G = I.gaussian_block(n, s, seed=1, complex_=(kind == "complex"))
    X = I.gaussian_block(n, s, seed=2, complex_=(kind == "complex"))
    out = pkg.sddmm(ctx, A, G, X, scale=-1.0)
    ref = O.sddmm(C.indptr, C.indices, G, X, scale=-1.0)
    np.testing.assert_allclose(out, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    A.close()


# ---------------------------------------------------------------- solver parity
def _problem(k):
    P = I.config(k, "small")
    if k == 3:   # unit-vector RHS break the BiCG/QMR families exactly (Lanczos breakdown); use Gaussian RHS
        B = I.gaussian_block(P.A.n, 12, seed=0, complex_=True)
        return P.A, B, P.name + "-gaussRHS"
    return P.A, P.B, P.name


CASES = [(k, m) for k in (1, 2, 3, 4, 5) for m in METHODS]


def _self_sensitivity(Acsr, B, method, ref, **kw):
    """The oracle's own spread: the same solve with B perturbed by 1e-15
    (relative, fixed seed).  Krylov recurrences amplify rounding differences,
    so two correct FP64 implementations can only agree to about this level."""
    rng = np.random.default_rng(12345)
    pert = B * (1 + 1e-15 * (rng.standard_normal(B.shape) if not np.iscomplexobj(B)
                             else rng.standard_normal(B.shape) + 1j * rng.standard_normal(B.shape)))
    r2 = O.solve(Acsr, pert, method, **kw)
    h = min(len(ref.history), len(r2.history))
    hist = np.abs(ref.history[:h] - r2.history[:h]) / ref.history[:h]
    return _rel(r2.X, ref.X), hist, abs(r2.iterations - ref.iterations)


@pytest.mark.parametrize("k,method", CASES)
def test_solve_matches_oracle(pkg, ctx, k, method):
    """Converged parity: same status, iteration count within 5% (plus the
    oracle's own spread), X within 100x the oracle's own sensitivity to 1e-15
    input perturbations (floor 1e-10), true residual at the stopping level."""
    Acsr, B, name = _problem(k)
    say("solve", name, method)
    ref = O.solve(Acsr, B, method, tol=1e-8, maxit=3000)
    xs, hs, its = _self_sensitivity(Acsr, B, method, ref, tol=1e-8, maxit=3000)
    A = pkg.Matrix.from_csr(ctx, Acsr)
    X, info = pkg.solve(ctx, A, B, method, tol=1e-8, maxit=3000)
    A.close()
    err = _rel(X, ref.X)
    say(f"  gpu status={info.status_name} it={info.iterations} res={info.rel_res_true:.3e} | "
        f"oracle status={ref.status} it={ref.iterations} res={ref.rel_res_true:.3e} | "
        f"err={err:.3e} oracle-self-spread={xs:.3e}")
    assert info.status == ref.status
    assert abs(info.iterations - ref.iterations) <= max(1, int(0.05 * ref.iterations)) + its
    assert info.matvecs * ref.iterations == ref.matvecs * info.iterations
    # the first iterations agree to rounding (before amplification sets in)
    m = min(8, len(ref.history), len(info.history))
    np.testing.assert_allclose(info.history[:m], ref.history[:m], rtol=1e-9, atol=0)
    # later iterations: within 100x the oracle's own spread
    m = min(50, len(ref.history), len(info.history), len(hs))
    d = np.abs(info.history[:m] - ref.history[:m]) / ref.history[:m]
    assert np.all(d <= np.maximum(1e-9, 100 * np.maximum.accumulate(hs[:m]))), (d.max(), hs[:m].max())
    assert err <= max(1e-10, 100 * xs), (err, xs)
    assert info.rel_res_true < 2e-8


@pytest.mark.parametrize("k,method", CASES)
def test_converged_to_1e12_matches_oracle(pkg, ctx, k, method):
    """Both sides run to a relative residual of 1e-12, where X is close to
    X* = A^{-1} B whatever the iteration path: same status, iteration count
    within 5% plus the oracle's own spread, and X within 1e-10 of the
    oracle's."""
    Acsr, B, name = _problem(k)
    say("solve 1e-12", name, method)
    ref = O.solve(Acsr, B, method, tol=1e-12, maxit=5000)
    xs, hs, its = _self_sensitivity(Acsr, B, method, ref, tol=1e-12, maxit=5000)
    A = pkg.Matrix.from_csr(ctx, Acsr)
    X, info = pkg.solve(ctx, A, B, method, tol=1e-12, maxit=5000)
    A.close()
    err = _rel(X, ref.X)
    say(f"  gpu status={info.status_name} it={info.iterations} res={info.rel_res_true:.3e} | "
        f"oracle status={ref.status} it={ref.iterations} (perturbed {ref.iterations + its} or "
        f"{ref.iterations - its}) | err={err:.3e} oracle-self-spread={xs:.3e}")
    assert info.status == ref.status == 0
    assert abs(info.iterations - ref.iterations) <= max(1, int(0.05 * ref.iterations)) + its
    assert err <= 1e-10, (err, xs)


@pytest.mark.parametrize("k,method", [(k, m) for k in (1, 2, 3, 4, 5) for m in METHODS])
def test_fixed_iterations_match_oracle(pkg, ctx, k, method):
    """Same number of iterations on both sides, on every workload family: the
    iterates agree to 1e-10."""
    Acsr, B, name = _problem(k)
    it = 8
    ref = O.solve(Acsr, B, method, tol=0.0, maxit=it)
    xs, hs, _ = _self_sensitivity(Acsr, B, method, ref, tol=0.0, maxit=it)
    A = pkg.Matrix.from_csr(ctx, Acsr)
    X, info = pkg.solve(ctx, A, B, method, tol=0.0, maxit=it)
    A.close()
    assert info.iterations == it and info.status == ref.status
    # 1e-10, or 100x the oracle's own spread where the recurrence amplifies
    # rounding faster (Bl-BiCG-rQ on the convection-dominated 3D problem)
    assert _rel(X, ref.X) < max(1e-10, 100 * xs), (_rel(X, ref.X), xs)
    np.testing.assert_allclose(info.history, ref.history, rtol=max(1e-10, 100 * hs.max()), atol=0)


@pytest.mark.parametrize("method", METHODS)
def test_adjoint_solve(pkg, ctx, method):
    """Adjoint solve A^H X = B (the same solver with the roles of the A and A^H
    operands swapped) against the oracle run on the explicit conjugate
    transpose, with the forward solve's criteria: same status, iterations within
    5% plus the oracle's own spread, history to rounding in the first
    iterations, X within max(1e-10, 100x the oracle's own spread)."""
    Acsr, B, name = _problem(4)
    At = Acsr.to_scipy().conj().T.tocsr()
    say("adjoint", name, method)
    ref = O.solve(At, B, method, tol=1e-8, maxit=3000)
    xs, hs, its = _self_sensitivity(At, B, method, ref, tol=1e-8, maxit=3000)
    A = pkg.Matrix.from_csr(ctx, Acsr)
    X, info = pkg.solve(ctx, A, B, method, tol=1e-8, maxit=3000, adjoint=True)
    A.close()
    err = _rel(X, ref.X)
    say(f"  gpu it={info.iterations} oracle it={ref.iterations} err={err:.3e} oracle-self-spread={xs:.3e}")
    assert info.status == ref.status == 0
    assert abs(info.iterations - ref.iterations) <= max(1, int(0.05 * ref.iterations)) + its
    m = min(8, len(ref.history), len(info.history))
    np.testing.assert_allclose(info.history[:m], ref.history[:m], rtol=1e-9, atol=0)
    assert err <= max(1e-10, 100 * xs), (err, xs)


MIXED_PARITY_TOL = 1e-11   # outer tolerance of the parity run (the timed runs use 1e-8)


@pytest.mark.parametrize("method", ["egl_bicg", "gl_bicgstab", "bl_bicgstab_rq", "egl_qmr", "bl_bicg_rq"])
@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_mixed_precision_refinement(pkg, ctx, k, method):
    """FP32 inner solves inside FP64 refinement.  The solve at the timing
    tolerance (1e-8) must reach it; the parity run tightens the outer
    tolerance and its X must be within 1e-8 of the oracle's X* (the FP64 oracle
    run to 1e-12).  Both errors are printed."""
    Acsr, B, name = _problem(k)
    say("mixed", name, method)
    ref = O.solve(Acsr, B, method, tol=1e-12, maxit=5000)
    assert ref.status == 0
    A = pkg.Matrix.from_csr(ctx, Acsr)
    X8, i8 = pkg.solve(ctx, A, B, method, tol=1e-8, precision="fp32_refine", inner_tol=1e-4, max_outer=20)
    X, info = pkg.solve(ctx, A, B, method, tol=MIXED_PARITY_TOL, precision="fp32_refine", inner_tol=1e-4,
                        max_outer=20)
    A.close()
    err8, err = _rel(X8, ref.X), _rel(X, ref.X)
    say(f"  tol 1e-8: status={i8.status_name} outer={i8.outer_iterations} (fp64 {i8.fp64_outer_iterations}) "
        f"inner_it={i8.iterations} res={i8.rel_res_true:.3e} err_vs_X*={err8:.3e}")
    say(f"  tol {MIXED_PARITY_TOL:g}: status={info.status_name} outer={info.outer_iterations} "
        f"(fp64 {info.fp64_outer_iterations}) inner_it={info.iterations} res={info.rel_res_true:.3e} "
        f"err_vs_X*={err:.3e}")
    assert i8.status == 0 and i8.rel_res_true <= 1e-8
    assert info.status == 0 and info.rel_res_true <= MIXED_PARITY_TOL
    assert err <= 1e-8, err


def test_sell_solve_matches_csr(pkg, ctx):
    Acsr, B, name = _problem(4)
    A1 = pkg.Matrix.from_csr(ctx, Acsr)
    A2 = pkg.Matrix.from_csr(ctx, Acsr, fmt="sell", sell_C=32, sell_sigma=256)
    for method in ("egl_bicg", "bl_bicgstab_rq"):
        X1, i1 = pkg.solve(ctx, A1, B, method)
        X2, i2 = pkg.solve(ctx, A2, B, method)
        assert i1.iterations == i2.iterations
        assert _rel(X2, X1) < 1e-10
    assert A2.sell_padding >= 1.0
    A1.close(); A2.close()


# ---------------------------------------------------------------- failure paths
def test_breakdown_zero_mean_shadow(pkg, ctx):
    C = I.convdiff2d(8)
    b = I.gaussian_block(C.n, 1, seed=18)
    B = np.hstack([b, -b])
    A = pkg.Matrix.from_csr(ctx, C)
    X, info = pkg.solve(ctx, A, B, "egl_bicg", preprocess_qr=False)
    assert info.status_name == "breakdown" and info.breakdown_iter == 0
    assert np.all(X == 0)
    A.close()


def test_not_converged_returns_last_iterate(pkg, ctx):
    C = I.convdiff2d(12)
    B = I.gaussian_block(C.n, 2, seed=21)
    ref = O.solve(C, B, "gl_bicg", tol=1e-8, maxit=3)
    A = pkg.Matrix.from_csr(ctx, C)
    X, info = pkg.solve(ctx, A, B, "gl_bicg", tol=1e-8, maxit=3)
    assert info.status_name == "not_converged" and info.iterations == 3 and len(info.history) == 4
    assert _rel(X, ref.X) < 1e-12
    A.close()


def test_nan_input_rejected(pkg, ctx):
    C = I.convdiff2d(8)
    B = I.gaussian_block(C.n, 2, seed=1)
    B[3, 1] = np.nan
    A = pkg.Matrix.from_csr(ctx, C)
    with pytest.raises(pkg.SkrError):
        pkg.solve(ctx, A, B, "gl_bicg")
    A.close()


def test_matrix_create_rejects_sizes_out_of_range(pkg, ctx):
    """Rejected before any array is read: n = 0, n above 2^31 - 2^20 (the row
    sweeps step int32 row indices past n), and SELL with C outside {16, 32, 64}."""
    import ctypes
    lib = pkg.load_library()
    rp = np.zeros(2, dtype=np.int64)
    ci = np.zeros(1, dtype=np.int32)
    va = np.zeros(1)
    from paper_1504_04395_amd import _binding as Bd
    f = Bd.skr_format_opts(0, 32, 256, 0)
    for n in (0, 2**31 - 2**20 + 1, 2**31):
        # straight through the C ABI: the binding would refuse the short indptr first
        h = ctypes.c_void_p()
        rc = lib.skr_matrix_create(ctx.handle, n, 0, rp.ctypes.data, ci.ctypes.data, va.ctypes.data, 0, 0,
                                   ctypes.byref(f), ctypes.byref(h))
        assert rc == Bd.SKR_E_INVALID and not h.value
        assert "n must be in" in lib.skr_last_error(ctx.handle).decode()
    with pytest.raises(pkg.SkrError, match="SELL needs C"):
        pkg.Matrix(ctx, 1, np.array([0, 1]), np.array([0], dtype=np.int32), np.ones(1), fmt="sell", sell_C=8,
                   sell_sigma=64)


def test_warm_start(pkg, ctx):
    C = I.convdiff2d(16)
    B = I.gaussian_block(C.n, 3, seed=2)
    A = pkg.Matrix.from_csr(ctx, C)
    X1, i1 = pkg.solve(ctx, A, B, "egl_bicg", tol=1e-4)
    X2, i2 = pkg.solve(ctx, A, B, "egl_bicg", X=X1.copy(), tol=1e-6)
    ref = O.solve(C, B, "egl_bicg", tol=1e-6, X0=X1)
    assert i2.status == 0 and abs(i2.iterations - ref.iterations) <= max(1, int(0.05 * ref.iterations))
    assert _rel(X2, ref.X) < 1e-8
    A.close()


def test_graph_and_eager_agree(pkg, ctx):
    Acsr, B, name = _problem(2)
    A = pkg.Matrix.from_csr(ctx, Acsr)
    for method in ("egl_qmr", "bl_bicg_rq"):
        X1, i1 = pkg.solve(ctx, A, B, method, use_graph=True)
        X2, i2 = pkg.solve(ctx, A, B, method, use_graph=False)
        X3, i3 = pkg.solve(ctx, A, B, method, use_graph=True)   # cached graph replay
        assert i1.iterations == i2.iterations == i3.iterations
        assert np.array_equal(X1, X2) and np.array_equal(X1, X3)
    A.close()


# ---------------------------------------------------------------- awkward block widths
@pytest.mark.parametrize("kind,s", [("real", 20), ("real", 31), ("complex", 17), ("complex", 25)])
@pytest.mark.parametrize("method", ["bl_bicg_rq", "bl_bicgstab_rq"])
def test_block_methods_at_odd_widths(pkg, ctx, kind, s, method):
    """Widths that leave padding columns in the MFMA row tiles (s not a multiple
    of 16) on a row count that leaves a ragged last tile: five iterations
    against the oracle."""
    if kind == "real":
        Acsr = I.convdiff2d(37, (20.0, 20.0))                      # n = 1369
    else:
        Acsr = I.powerlaw(1500 + 7, seed=5, lo=4, hi=30, mean=8.0)
    B = I.gaussian_block(Acsr.n, s, seed=s, complex_=(kind == "complex"))
    it = 5
    ref = O.solve(Acsr, B, method, tol=0.0, maxit=it)
    spread, hs, _ = _self_sensitivity(Acsr, B, method, ref, tol=0.0, maxit=it)
    A = pkg.Matrix.from_csr(ctx, Acsr)
    X, info = pkg.solve(ctx, A, B, method, tol=0.0, maxit=it)
    A.close()
    err = _rel(X, ref.X)
    print(f"{method} {kind} s={s} n={Acsr.n}: err={err:.2e} spread={spread:.2e}", flush=True)
    assert info.status == ref.status and info.iterations == it
    assert err < max(1e-10, 100 * spread)
    np.testing.assert_allclose(info.history, ref.history, rtol=max(1e-9, 100 * hs.max()), atol=0)
