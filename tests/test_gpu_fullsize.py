"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark uses: sampled outputs the oracle computes row by row, iterates after
a few iterations against the oracle, and properties that hold at any size
(true residual recomputed on the CPU)."""
import os
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


def _sampled_rows_ok(Acsr, X, Y, nsample=3000, seed=0):
    rng = np.random.default_rng(seed)
    rows = np.concatenate([rng.choice(Acsr.n, nsample, replace=False), [0, Acsr.n - 1]])
    S = Acsr.to_scipy()
    ref = S[rows] @ X
    scale = np.abs(ref).max()
    np.testing.assert_allclose(Y[rows], ref, rtol=0, atol=1e-13 * scale)


@pytest.fixture(scope="module")
def cfg2():
    return I.config(2)            # 3D convection-diffusion 128^3, s = 16


def test_spmm_full_convdiff3d(env, cfg2):
    P, ctx = env
    import torch
    say("spmm full 128^3")
    A = P.Matrix.from_csr(ctx, cfg2.A)
    X = torch.from_numpy(cfg2.B).cuda()
    for adj in (False, True):
        Y = P.spmm(ctx, A, X, adjoint=adj).cpu().numpy()
        Aref = cfg2.A if not adj else _transpose(cfg2.A)
        _sampled_rows_ok(Aref, cfg2.B, Y)
    A.close()


def _transpose(C):
    S = C.to_scipy().conj().T.tocsr()
    S.sort_indices()
    return I.CSR(C.n, S.indptr.astype(np.int64), S.indices.astype(np.int32), S.data)


@pytest.mark.parametrize("method", ["bl_bicg_rq", "egl_qmr", "bl_bicgstab_rq"])
def test_first_iterations_full_convdiff3d(env, cfg2, method):
    """Three iterations at full size on both sides: iterates agree to 1e-10."""
    P, ctx = env
    import torch
    say("3 iterations full 128^3", method)
    ref = O.solve(cfg2.A, cfg2.B, method, tol=0.0, maxit=3)
    A = P.Matrix.from_csr(ctx, cfg2.A)
    X, info = P.solve(ctx, A, torch.from_numpy(cfg2.B).cuda(), method, tol=0.0, maxit=3)
    A.close()
    X = X.cpu().numpy()
    err = np.linalg.norm(X - ref.X) / np.linalg.norm(ref.X)
    say(f"  err {err:.2e}")
    assert info.iterations == 3 and err < 1e-10
    np.testing.assert_allclose(info.history, ref.history, rtol=1e-10)


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden_runs(grid=128):
    """{method: {seed: (status, iterations)}} of the oracle's runs on the
    benchmark workload (tests/golden/make_fullsize_counts.py)."""
    out = {}
    for line in open(os.path.join(GOLDEN, "fullsize_iterations.txt")):
        f = line.split()
        if f and not f[0].startswith("#") and int(f[0]) == grid:
            out.setdefault(f[1], {})[int(f[2])] = (int(f[3]), int(f[4]))
    return out


@pytest.mark.parametrize("method", ["bl_bicg_rq", "egl_qmr", "bl_bicgstab_rq"])
def test_fullsize_iteration_count(env, cfg2, method):
    """The benchmark's own solves, in its launch configuration (tol 1e-8, at
    most 1200 iterations).  Where the oracle's run on the inputs themselves
    converged: the GPU's iteration count within 5% of it, plus the spread of
    the oracle's converged counts over runs with B perturbed by 1e-15.  Where
    it did not (Bl-BiCG-rQ on this input runs to the cap with a growing
    residual, while its 1e-15-perturbed copies converge): the GPU must
    converge, with a count inside the range of the oracle's converged
    perturbed runs widened by 5%."""
    P, ctx = env
    import torch
    runs = _golden_runs().get(method, {})
    if 0 not in runs:
        pytest.skip(f"no oracle count on file for {method} (make_fullsize_counts.py --method {method})")
    conv = sorted(it for st, it in runs.values() if st == 0)
    A = P.Matrix.from_csr(ctx, cfg2.A)
    X, info = P.solve(ctx, A, torch.from_numpy(cfg2.B).cuda(), method, tol=1e-8, maxit=1200)
    A.close()
    st0, it0 = runs[0]
    say(f"full 128^3 {method}: gpu it={info.iterations} status={info.status_name} | oracle on B: status={st0} "
        f"it={it0} | converged oracle counts {conv}")
    assert info.status == 0
    if st0 == 0:
        spread = max(conv) - min(conv)
        assert abs(info.iterations - it0) <= max(1, int(0.05 * it0)) + spread
    else:
        assert len(conv) >= 2, "too few converged oracle runs on file"
        lo, hi = min(conv), max(conv)
        assert lo - max(1, int(0.05 * lo)) <= info.iterations <= hi + max(1, int(0.05 * hi))


def _xstar_rows():
    rows, vals = [], []
    for line in open(os.path.join(GOLDEN, "fullsize_xstar_rows.txt")):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows.append(int(f[0]))
        vals.append([float(v) for v in f[1:]])
    return np.array(rows), np.array(vals)


def test_mixed_full_convdiff3d_against_xstar(env, cfg2):
    """FP32 inner solves inside FP64 refinement on the full benchmark workload:
    at the timing tolerance 1e-8 the true residual (recomputed on the CPU) is
    met; the parity run tightens the outer tolerance to 1e-12 and its X agrees
    with the oracle's X* (eGl-QMR to 1e-12) to 1e-8 on the sampled rows."""
    P, ctx = env
    import torch
    rows, xs = _xstar_rows()
    A = P.Matrix.from_csr(ctx, cfg2.A)
    Bd = torch.from_numpy(cfg2.B).cuda()
    S = cfg2.A.to_scipy()
    for tol in (1e-8, 1e-12):
        X, info = P.solve(ctx, A, Bd, "egl_qmr", tol=tol, precision="fp32_refine", max_outer=20)
        X = X.cpu().numpy()
        rel = np.linalg.norm(cfg2.B - S @ X) / np.linalg.norm(cfg2.B)
        err = np.linalg.norm(X[rows] - xs) / np.linalg.norm(xs)
        say(f"  mixed egl_qmr tol={tol:g}: status={info.status_name} outer={info.outer_iterations} "
            f"inner it={info.iterations} true_res_cpu={rel:.2e} err_vs_X*(sampled rows)={err:.2e}")
        assert info.status == 0 and rel <= 1.5 * tol
        if tol <= 1e-12:
            assert err <= 1e-8, err
    A.close()


@pytest.mark.parametrize("method,precision", [("egl_qmr", "fp64"), ("bl_bicgstab_rq", "fp64"),
                                              ("egl_qmr", "fp32_refine")])
def test_solve_full_convdiff3d(env, cfg2, method, precision):
    """Converged full-size solve: the true residual, recomputed on the CPU with
    the oracle's sparse product, is at the 1e-8 level."""
    P, ctx = env
    import torch
    say("solve full 128^3", method, precision)
    A = P.Matrix.from_csr(ctx, cfg2.A)
    X, info = P.solve(ctx, A, torch.from_numpy(cfg2.B).cuda(), method, tol=1e-8, precision=precision)
    A.close()
    X = X.cpu().numpy()
    S = cfg2.A.to_scipy()
    rel = np.linalg.norm(cfg2.B - S @ X) / np.linalg.norm(cfg2.B)
    say(f"  status={info.status_name} it={info.iterations} outer={info.outer_iterations} "
        f"true_res_gpu={info.rel_res_true:.2e} true_res_cpu={rel:.2e}")
    assert info.status == 0
    assert abs(rel - info.rel_res_true) <= 1e-3 * rel + 1e-15
    assert rel < 1.5e-8


def test_powerlaw_full_sell_vs_csr(env):
    """Random power-law matrix, n = 2^20, s = 32 complex: SELL-C-sigma and CSR
    products against sampled rows, and a converged eGl-BiCG solve."""
    P, ctx = env
    import torch
    prob = I.config(4)
    say("powerlaw full", prob.A.nnz)
    Ac = P.Matrix.from_csr(ctx, prob.A)
    As = P.Matrix.from_csr(ctx, prob.A, fmt="sell", sell_C=32, sell_sigma=256)
    say("  sell padding", As.sell_padding)
    Xd = torch.from_numpy(prob.B).cuda()
    Yc = P.spmm(ctx, Ac, Xd).cpu().numpy()
    Ys = P.spmm(ctx, As, Xd).cpu().numpy()
    _sampled_rows_ok(prob.A, prob.B, Yc)
    _sampled_rows_ok(prob.A, prob.B, Ys)
    X, info = P.solve(ctx, As, Xd, "egl_bicg", tol=1e-8)
    X = X.cpu().numpy()
    rel = np.linalg.norm(prob.B - prob.A.to_scipy() @ X) / np.linalg.norm(prob.B)
    say(f"  egl_bicg sell: it={info.iterations} res={rel:.2e}")
    assert info.status == 0 and rel < 1.5e-8
    Ac.close()
    As.close()


def test_wilson_full_bicgstab_rq(env):
    """Wilson-type operator on 16^4 x 12 (n = 786,432, 49 nonzeros per row),
    unit right-hand sides: Bl-BiCGStab-rQ, FP64 and FP32 + refinement."""
    P, ctx = env
    import torch
    prob = I.config(3)
    say("wilson full", prob.A.n, prob.A.nnz)
    A = P.Matrix.from_csr(ctx, prob.A)
    Bd = torch.from_numpy(prob.B).cuda()
    Y = P.spmm(ctx, A, Bd).cpu().numpy()
    _sampled_rows_ok(prob.A, prob.B, Y)
    S = prob.A.to_scipy()
    for precision in ("fp64", "fp32_refine"):
        X, info = P.solve(ctx, A, Bd, "bl_bicgstab_rq", tol=1e-8, precision=precision)
        X = X.cpu().numpy()
        rel = np.linalg.norm(prob.B - S @ X) / np.linalg.norm(prob.B)
        say(f"  {precision}: status={info.status_name} it={info.iterations} res={rel:.2e}")
        assert info.status == 0 and rel < 1.5e-8
    A.close()


def test_block_fp32_inner_failure_falls_back(env, cfg2):
    """On the full 3D problem the block method's FP32 inner solve diverges (its
    s x s coefficient systems reach condition numbers near 1e5, which FP32
    block data cannot support).  The refinement stops that inner solve early,
    redoes the step in FP64, reports how many steps it redid, and converges."""
    P, ctx = env
    import torch
    A = P.Matrix.from_csr(ctx, cfg2.A)
    X, info = P.solve(ctx, A, torch.from_numpy(cfg2.B).cuda(), "bl_bicgstab_rq", tol=1e-8,
                      precision="fp32_refine", maxit=2000)
    A.close()
    X = X.cpu().numpy()
    rel = np.linalg.norm(cfg2.B - cfg2.A.to_scipy() @ X) / np.linalg.norm(cfg2.B)
    say(f"  bl_bicgstab_rq fp32_refine: status={info.status_name} outer={info.outer_iterations} "
        f"fp64 steps={info.fp64_outer_iterations} it={info.iterations} res={rel:.2e}")
    assert info.status == 0 and rel < 1.5e-8
    assert 0 <= info.fp64_outer_iterations <= info.outer_iterations
