"""CPU-only: the Python binding rejects operands whose shape, element type or
memory kind does not match the matrix before it calls the library, so a short
or mistyped buffer never reaches a C call that would read or write n x s
elements through it."""
import types

import numpy as np
import pytest

from paper_1504_04395_amd import _binding as B


class _NoCalls:
    """Stands in for the loaded library: any C call fails the test."""

    def __getattr__(self, name):
        raise AssertionError(f"library function {name} called despite invalid arguments")


@pytest.fixture()
def nolib(monkeypatch):
    monkeypatch.setattr(B, "load_library", lambda *a, **k: _NoCalls())
    ctx = types.SimpleNamespace(handle=None)
    real = types.SimpleNamespace(ctx=ctx, handle=None, n=10, nnz=28, dtype=B.SKR_F64, version=0)
    cplx = types.SimpleNamespace(ctx=ctx, handle=None, n=10, nnz=28, dtype=B.SKR_C64, version=0)
    return ctx, real, cplx


def _blk(n, s, dt=np.float64):
    return np.zeros((n, s), dtype=dt)


@pytest.mark.parametrize("bad", ["short_B", "wide_B", "B_1d", "B_int", "B_complex_for_real",
                                 "X_short", "X_shape", "X_dtype"])
def test_solve_rejects(nolib, bad):
    ctx, A, _ = nolib
    Bm, X = _blk(10, 3), None
    if bad == "short_B":
        Bm = _blk(9, 3)
    elif bad == "wide_B":
        Bm = _blk(10, 33)
    elif bad == "B_1d":
        Bm = np.zeros(10)
    elif bad == "B_int":
        Bm = np.zeros((10, 3), dtype=np.int64)
    elif bad == "B_complex_for_real":
        Bm = _blk(10, 3, np.complex128)
    elif bad == "X_short":
        X = _blk(9, 3)
    elif bad == "X_shape":
        X = _blk(10, 2)
    elif bad == "X_dtype":
        X = _blk(10, 3, np.complex128)
    with pytest.raises(ValueError):
        B.solve(ctx, A, Bm, "gl_bicg", X=X)


def test_complex_matrix_rejects_real_block(nolib):
    ctx, _, A = nolib
    with pytest.raises(ValueError, match="complex128"):
        B.solve(ctx, A, _blk(10, 2), "egl_bicg")
    with pytest.raises(ValueError, match="complex128"):
        B.spmm(ctx, A, _blk(10, 2))


@pytest.mark.parametrize("fn", ["spmm", "precond_apply"])
def test_products_reject(nolib, fn):
    ctx, A, _ = nolib
    f = getattr(B, fn)
    with pytest.raises(ValueError):
        f(ctx, A, _blk(11, 4))                    # wrong row count
    with pytest.raises(ValueError):
        f(ctx, A, _blk(10, 4), _blk(10, 3))       # output of another shape
    with pytest.raises(ValueError):
        f(ctx, A, _blk(10, 4), _blk(10, 4, np.complex128))


def test_sddmm_rejects(nolib):
    ctx, A, _ = nolib
    with pytest.raises(ValueError):
        B.sddmm(ctx, A, _blk(10, 4), _blk(10, 3))            # G and X differ
    with pytest.raises(ValueError):
        B.sddmm(ctx, A, _blk(9, 4), _blk(9, 4))              # wrong row count
    with pytest.raises(ValueError):
        B.sddmm(ctx, A, _blk(10, 4), _blk(10, 4), out=np.zeros(27))   # out shorter than nnz
    with pytest.raises(ValueError):
        B.sddmm(ctx, A, _blk(10, 4), _blk(10, 4), out=np.zeros(28, dtype=np.complex128))


def test_update_values_rejects(nolib):
    ctx, A, _ = nolib
    M = B.Matrix.__new__(B.Matrix)
    M.__dict__.update(ctx=ctx, handle=None, n=A.n, nnz=A.nnz, dtype=A.dtype, version=0)
    with pytest.raises(ValueError):
        M.update_values(np.zeros(27))
    with pytest.raises(ValueError):
        M.update_values(np.zeros(28, dtype=np.complex128))
    assert M.version == 0


def test_matrix_create_rejects_host_arrays(nolib):
    ctx, _, _ = nolib
    rp = np.array([0, 1, 2], dtype=np.int64)
    with pytest.raises(ValueError, match="n \\+ 1"):
        B.Matrix(ctx, 3, rp, np.array([0, 1], dtype=np.int32), np.ones(2))
    with pytest.raises(ValueError, match="indptr\\[n\\]"):
        B.Matrix(ctx, 2, rp, np.array([0], dtype=np.int32), np.ones(2))
    with pytest.raises(ValueError, match="float64 or complex128"):
        B.Matrix(ctx, 2, rp, np.array([0, 1], dtype=np.int32), np.ones(2, dtype=np.float32))


def test_matrix_create_rejects_torch_index_types(nolib):
    torch = pytest.importorskip("torch")
    ctx, _, _ = nolib
    rp = torch.tensor([0, 1, 2], dtype=torch.int64)
    ci = torch.tensor([0, 1], dtype=torch.int32)
    va = torch.ones(2, dtype=torch.float64)
    with pytest.raises(ValueError, match="int64"):
        B.Matrix(ctx, 2, rp.to(torch.int32), ci, va)
    with pytest.raises(ValueError, match="int32"):
        B.Matrix(ctx, 2, rp, ci.to(torch.int64), va)
    with pytest.raises(ValueError, match="n \\+ 1"):
        B.Matrix(ctx, 3, rp, ci, va)
    with pytest.raises(ValueError, match="nnz"):
        B.Matrix(ctx, 2, rp, ci, torch.ones(3, dtype=torch.float64))
    with pytest.raises(ValueError, match="float64 or complex128"):
        B.Matrix(ctx, 2, rp, ci, va.to(torch.float32))
