"""GPU: differentiable solve (adjoint solve + SDDMM) against the dense-LU
reference gradient and central finite differences."""
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
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1504_04395_amd as P
    ctx = P.Context(0)
    yield P, ctx
    ctx.close()


def _loss_and_grads(P, ctx, Acsr, B, Xt, method, precision, tol):
    import torch
    M = P.Matrix.from_csr(ctx, Acsr)
    vals = torch.tensor(Acsr.data, dtype=torch.float64, device="cuda", requires_grad=True)
    Bt = torch.tensor(B, dtype=torch.float64, device="cuda", requires_grad=True)
    Xtt = torch.tensor(Xt, dtype=torch.float64, device="cuda")
    X = P.sparse_solve(vals, Bt, M, method, tol, precision)
    L = ((X - Xtt) ** 2).sum()
    L.backward()
    out = (L.item(), vals.grad.cpu().numpy(), Bt.grad.cpu().numpy(), X.detach().cpu().numpy())
    M.close()
    return out


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
def test_gradient_matches_dense_lu(env, precision):
    P, ctx = env
    prob = I.config(5, "small")                       # 2D 64 x 64 convection-diffusion, s = 8
    A, B, Xt = prob.A, prob.B, prob.extra["X_target"]
    L, gv, gB, X = _loss_and_grads(P, ctx, A, B, Xt, "egl_bicg", precision, 1e-11)
    Ad = A.to_scipy().toarray()
    Xd = np.linalg.solve(Ad, B)
    Xr, GBr, GAr = O.dense_solve_grad(Ad, B, 2 * (Xd - Xt))
    rows = np.repeat(np.arange(A.n), np.diff(A.indptr))
    gv_ref = GAr[rows, A.indices]
    say(precision, "grad_vals rel err", np.linalg.norm(gv - gv_ref) / np.linalg.norm(gv_ref),
        "grad_B rel err", np.linalg.norm(gB - GBr) / np.linalg.norm(GBr))
    assert np.linalg.norm(X - Xr) / np.linalg.norm(Xr) < 1e-8
    assert np.linalg.norm(gv - gv_ref) / np.linalg.norm(gv_ref) < 1e-6
    assert np.linalg.norm(gB - GBr) / np.linalg.norm(GBr) < 1e-6


def test_two_solves_share_one_matrix(env):
    """Two forward solves with different values on one Matrix, then one backward
    pass through both: each solve's gradient must use its own A (the second
    forward pass overwrote the matrix's values before the first backward)."""
    import torch
    P, ctx = env
    prob = I.config(5, "small")
    A, B, Xt = prob.A, prob.B, prob.extra["X_target"]
    vals2 = A.data * 1.25 + 0.01 * np.random.default_rng(7).standard_normal(A.nnz) * (A.data != 0)
    M = P.Matrix.from_csr(ctx, A)
    v1 = torch.tensor(A.data, device="cuda", requires_grad=True)
    v2 = torch.tensor(vals2, device="cuda", requires_grad=True)
    Bt = torch.tensor(B, device="cuda", requires_grad=True)
    Xtt = torch.tensor(Xt, device="cuda")
    X1 = P.sparse_solve(v1, Bt, M, "egl_bicg", 1e-11, "fp64")
    X2 = P.sparse_solve(v2, Bt, M, "egl_bicg", 1e-11, "fp64")
    L = ((X1 - Xtt) ** 2).sum() + 0.5 * ((X2 - Xtt) ** 2).sum()
    L.backward()
    M.close()
    rows = np.repeat(np.arange(A.n), np.diff(A.indptr))
    gB_ref = np.zeros_like(B)
    for vals, w, g in ((A.data, 1.0, v1.grad), (vals2, 0.5, v2.grad)):
        Ad = A.to_scipy().toarray()
        Ad[rows, A.indices] = vals
        Xd = np.linalg.solve(Ad, B)
        _, GBr, GAr = O.dense_solve_grad(Ad, B, 2 * w * (Xd - Xt))
        gv_ref = GAr[rows, A.indices]
        err = np.linalg.norm(g.cpu().numpy() - gv_ref) / np.linalg.norm(gv_ref)
        say("two solves, one matrix: grad_vals rel err", err)
        assert err < 1e-6
        gB_ref += GBr
    assert np.linalg.norm(Bt.grad.cpu().numpy() - gB_ref) / np.linalg.norm(gB_ref) < 1e-6


@pytest.mark.parametrize("precision", ["fp64", "fp32_refine"])
@pytest.mark.parametrize("grid", [64, 1024])
def test_gradient_matches_finite_differences(env, grid, precision):
    """Central differences of L with solves at 1e-12.  With FP32 inner solves
    on the 1024 x 1024 grid the outer FP64 refinement targets 1e-11: on that
    adjoint system it stagnates near 3e-12 (30 outer steps measured), and 1e-11
    still leaves the solve error far below the 1e-6 bar there (on the 64 x 64
    grid 1e-11 is not enough for the A direction: best step 1.4e-6).  Along F (on B) central
    differences are exact, since L is quadratic in B.  Along E (on A's stored
    values) the step is swept over relative sizes 1e-7..1e-10 (kappa(A) grows
    like the grid size squared, so a larger step leaves the linear regime);
    the best agreement must be within 1e-6."""
    import torch
    P, ctx = env
    A = I.convdiff2d(grid, (20.0, 20.0))
    B = I.gaussian_block(A.n, 8, seed=0)
    Xt = I.gaussian_block(A.n, 8, seed=1)
    rng = np.random.default_rng(3)
    E = rng.standard_normal(A.nnz)
    F = rng.standard_normal(B.shape)
    tol = 1e-11 if (precision == "fp32_refine" and grid >= 1024) else 1e-12
    L0, gv, gB, _ = _loss_and_grads(P, ctx, A, B, Xt, "egl_bicg", precision, tol)
    M = P.Matrix.from_csr(ctx, A)
    Xtt = torch.tensor(Xt, device="cuda")

    def loss(hE, hF):
        vals = torch.tensor(A.data + hE * E, device="cuda")
        Bt = torch.tensor(B + hF * F, device="cuda")
        X = P.sparse_solve(vals, Bt, M, "egl_bicg", tol, precision)
        return float(((X - Xtt) ** 2).sum())

    hF = 1e-3 * np.linalg.norm(B) / np.linalg.norm(F)
    fdF = (loss(0.0, hF) - loss(0.0, -hF)) / (2 * hF)
    anF = float(np.sum(gB * F))
    relF = abs(fdF - anF) / abs(anF)
    anE = float(gv @ E)
    relE = []
    for r in (1e-7, 1e-8, 1e-9, 1e-10):
        hE = r * np.linalg.norm(A.data) / np.linalg.norm(E)
        fdE = (loss(hE, 0.0) - loss(-hE, 0.0)) / (2 * hE)
        relE.append(abs(fdE - anE) / abs(anE))
    M.close()
    say(f"grid {grid} {precision}: F direction rel {relF:.2e}; E direction rel over steps 1e-7..1e-10: "
        + ", ".join(f"{x:.1e}" for x in relE))
    assert relF <= 1e-6
    assert min(relE) <= 1e-6
