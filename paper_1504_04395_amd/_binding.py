"""ctypes binding of the C ABI declared in include/skrylov.h.

Argument marshalling only: every arithmetic step runs in the HIP library.  The
names mirror the C functions (``skr_solve`` -> :func:`solve`, ...).  Blocks are
row-major n x s arrays: numpy arrays (host memory) or torch CUDA tensors (device
memory, used in place).  Real data are float64, complex data complex128.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libskrylov.so")

SKR_OK, SKR_E_INVALID, SKR_E_ALLOC, SKR_E_HIP, SKR_E_UNSUPPORTED = 0, -1, -2, -3, -4
SKR_NOT_CONVERGED, SKR_BREAKDOWN, SKR_DIVERGED = 1, 2, 3
STATUS_NAMES = {0: "ok", 1: "not_converged", 2: "breakdown", 3: "diverged",
                -1: "invalid", -2: "alloc", -3: "hip", -4: "unsupported"}
PRECONDS = {None: 0, "none": 0, "ilu0": 1}
METHODS = {"gl_bicg": 0, "egl_bicg": 1, "gl_qmr": 2, "egl_qmr": 3, "gl_bicgstab": 4,
           "bl_bicg_rq": 5, "bl_bicgstab_rq": 6, "bl_bicg": 7, "bl_bicgstab": 8, "li_bicg": 9,
           "li_bicgstab": 10, "li_qmr": 11}
SKR_F64, SKR_C64 = 0, 1
SKR_MEM_HOST, SKR_MEM_DEVICE = 0, 1
SKR_FMT_CSR, SKR_FMT_SELL = 0, 1
PRECISIONS = {"fp64": 0, "fp32_refine": 1}


class skr_opts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("maxit", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("max_outer", ctypes.c_int32), ("preprocess_qr", ctypes.c_int32),
                ("zero_x0", ctypes.c_int32), ("check_every", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("fused_small", ctypes.c_int32)]


class skr_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iterations", ctypes.c_int32), ("matvecs", ctypes.c_int64),
                ("outer_iterations", ctypes.c_int32), ("breakdown_iter", ctypes.c_int32),
                ("rel_res_recursive", ctypes.c_double), ("rel_res_true", ctypes.c_double),
                ("history", ctypes.POINTER(ctypes.c_double)), ("history_cap", ctypes.c_int32),
                ("history_len", ctypes.c_int32), ("fp64_outer_iterations", ctypes.c_int32),
                ("single_workgroup", ctypes.c_int32)]


class skr_format_opts(ctypes.Structure):
    _fields_ = [("format", ctypes.c_int32), ("sell_C", ctypes.c_int32), ("sell_sigma", ctypes.c_int32),
                ("make_fp32", ctypes.c_int32)]


_VP = ctypes.c_void_p
_SIGS = {
    "skr_opts_default": (None, [ctypes.POINTER(skr_opts)]),
    "skr_context_create": (ctypes.c_int, [ctypes.c_int, _VP, ctypes.POINTER(_VP)]),
    "skr_context_destroy": (ctypes.c_int, [_VP]),
    "skr_context_set_stream": (ctypes.c_int, [_VP, _VP]),
    "skr_last_error": (ctypes.c_char_p, [_VP]),
    "skr_matrix_create": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int64, _VP, _VP, _VP, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.POINTER(skr_format_opts), ctypes.POINTER(_VP)]),
    "skr_matrix_update_values": (ctypes.c_int, [_VP, _VP, ctypes.c_int32]),
    "skr_matrix_destroy": (ctypes.c_int, [_VP]),
    "skr_matrix_sell_padding": (ctypes.c_double, [_VP]),
    "skr_solve": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, ctypes.c_int64, _VP, ctypes.c_int64, ctypes.c_int32,
                                 ctypes.c_int32, ctypes.POINTER(skr_opts), ctypes.c_int32, ctypes.POINTER(skr_result)]),
    "skr_spmm": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, ctypes.c_int64, _VP, ctypes.c_int64, ctypes.c_int32,
                                ctypes.c_int32]),
    "skr_sddmm": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int32]),
    "skr_matrix_ilu0": (ctypes.c_int, [_VP, _VP]),
    "skr_precond_apply": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, _VP, ctypes.c_int64, _VP, ctypes.c_int64,
                                         ctypes.c_int32, ctypes.c_int32]),
    "skr_block_qr": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _VP, _VP,
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_int32]),
    "skr_block_qr_noalloc": (ctypes.c_int, [_VP, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, _VP, _VP,
                                            ctypes.POINTER(ctypes.c_double)]),
}

_lib = None


def load_library(path: str = LIB_PATH):
    """Load libskrylov.so (built by ``python -m paper_1504_04395_amd.build``).  Raises if the
    library is missing: there is no fallback implementation."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing (run python -m paper_1504_04395_amd.build)")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class SkrError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def _check(ctx, rc):
    if rc < 0:
        msg = load_library().skr_last_error(ctx.handle if ctx is not None else None)
        raise SkrError(rc, msg.decode() if msg else "")
    return rc


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _order_torch(*xs):
    """Wait for torch's current stream when any argument is a CUDA tensor, so
    that the library's stream sees finished inputs."""
    for x in xs:
        if _is_torch(x) and x.is_cuda:
            import torch
            torch.cuda.current_stream().synchronize()
            return True
    return False


def _ptr_mem(x):
    """(pointer, mem kind, dtype code, keepalive)."""
    if _is_torch(x):
        import torch
        if not x.is_contiguous():
            raise ValueError("tensor must be contiguous")
        dt = SKR_C64 if x.dtype == torch.complex128 else SKR_F64
        if x.dtype not in (torch.float64, torch.complex128):
            raise ValueError("tensors must be float64 or complex128")
        return x.data_ptr(), (SKR_MEM_DEVICE if x.is_cuda else SKR_MEM_HOST), dt, x
    a = np.ascontiguousarray(x)
    if a.dtype == np.complex128:
        dt = SKR_C64
    elif a.dtype == np.float64:
        dt = SKR_F64
    else:
        raise ValueError("arrays must be float64 or complex128")
    return a.ctypes.data, SKR_MEM_HOST, dt, a


def _dtype_code(x):
    """SKR_F64 / SKR_C64 of a float64 / complex128 array or tensor, else None."""
    if _is_torch(x):
        import torch
        return {torch.float64: SKR_F64, torch.complex128: SKR_C64}.get(x.dtype)
    return {np.dtype(np.float64): SKR_F64, np.dtype(np.complex128): SKR_C64}.get(np.asarray(x).dtype)


def _check_block(x, n: int, dt: int, name: str, like=None):
    """Reject, before any library call, an operand whose shape or element type
    does not match what the C call will read or write: a 2-D block of n rows
    and 1..32 columns of A's element type, with the shape of ``like`` if given."""
    if len(x.shape) != 2:
        raise ValueError(f"{name} must be a 2-D n x s block")
    if int(x.shape[0]) != n:
        raise ValueError(f"{name} has {int(x.shape[0])} rows; the matrix has n = {n}")
    if not 1 <= int(x.shape[1]) <= 32:
        raise ValueError(f"{name} must have between 1 and 32 columns")
    if _dtype_code(x) != dt:
        raise ValueError(f"{name} must be {'complex128' if dt == SKR_C64 else 'float64'}, like the matrix")
    if like is not None and tuple(x.shape) != tuple(like.shape):
        raise ValueError(f"{name} must have the shape {tuple(like.shape)}")


class Context:
    """skr_context_create / skr_context_destroy."""

    def __init__(self, device: int = 0, stream=None):
        lib = load_library()
        h = _VP()
        rc = lib.skr_context_create(device, _VP(stream) if stream else None, ctypes.byref(h))
        if rc != 0:
            raise SkrError(rc, "context creation failed")
        self.handle = h

    def set_stream(self, stream):
        _check(self, load_library().skr_context_set_stream(self.handle, _VP(stream) if stream else None))

    def close(self):
        if getattr(self, "handle", None):
            load_library().skr_context_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Matrix:
    """skr_matrix_create from CSR arrays (indptr int64, indices int32, data
    float64/complex128) in host (numpy) or device (torch) memory."""

    def __init__(self, ctx: Context, n: int, indptr, indices, data, fmt: str = "csr", sell_C: int = 32,
                 sell_sigma: int = 256, make_fp32: bool = False):
        lib = load_library()
        self.ctx = ctx
        if _is_torch(data):
            import torch
            if not (_is_torch(indptr) and _is_torch(indices)):
                raise ValueError("indptr, indices and data must all be torch tensors, or all host arrays")
            if indptr.dtype != torch.int64 or indices.dtype != torch.int32:
                raise ValueError("indptr must be int64 and indices int32")
            if data.dtype not in (torch.float64, torch.complex128):
                raise ValueError("values must be float64 or complex128")
            if not (indptr.device == indices.device == data.device):
                raise ValueError("indptr, indices and data must live on the same device")
            if not (indptr.is_contiguous() and indices.is_contiguous() and data.is_contiguous()):
                raise ValueError("tensors must be contiguous")
            if indptr.dim() != 1 or int(indptr.numel()) != int(n) + 1:
                raise ValueError("indptr must have n + 1 entries")
            if indices.dim() != 1 or data.dim() != 1 or int(indices.numel()) != int(data.numel()):
                raise ValueError("indices and data must be 1-D with nnz entries each")
            p_rp, p_ci, p_va = indptr.data_ptr(), indices.data_ptr(), data.data_ptr()
            mem = SKR_MEM_DEVICE if data.is_cuda else SKR_MEM_HOST
            dtype = SKR_C64 if data.dtype == torch.complex128 else SKR_F64
            nnz = int(indices.numel())
            self._keep = [indptr, indices, data]
        else:
            rp = np.ascontiguousarray(indptr, dtype=np.int64)
            ci = np.ascontiguousarray(indices, dtype=np.int32)
            va = np.ascontiguousarray(data)
            if va.dtype not in (np.float64, np.complex128):
                raise ValueError("values must be float64 or complex128")
            if rp.ndim != 1 or rp.size != int(n) + 1:
                raise ValueError("indptr must have n + 1 entries")
            if ci.ndim != 1 or va.ndim != 1 or ci.size < int(rp[-1]) or va.size < int(rp[-1]) or int(rp[-1]) < 0:
                raise ValueError("indices and data must hold indptr[n] entries")
            self._keep = [rp, ci, va]
            p_rp, p_ci, p_va = rp.ctypes.data, ci.ctypes.data, va.ctypes.data
            mem = SKR_MEM_HOST
            dtype = SKR_C64 if np.iscomplexobj(va) else SKR_F64
            nnz = int(rp[-1])
        self.n = int(n)
        self.nnz = nnz
        self.dtype = dtype
        self.version = 0          # bumped by update_values (autograd checks it)
        f = skr_format_opts(SKR_FMT_SELL if fmt == "sell" else SKR_FMT_CSR, sell_C, sell_sigma, int(make_fp32))
        h = _VP()
        _check(ctx, lib.skr_matrix_create(ctx.handle, self.n, nnz, _VP(p_rp), _VP(p_ci), _VP(p_va), dtype, mem,
                                          ctypes.byref(f), ctypes.byref(h)))
        self.handle = h
        self._keep = []

    @classmethod
    def from_csr(cls, ctx, csr, **kw):
        """From an object with n, indptr, indices, data (e.g. inputs.CSR)."""
        return cls(ctx, csr.n, csr.indptr, csr.indices, csr.data, **kw)

    def update_values(self, data):
        if len(data.shape) != 1 or int(data.shape[0]) != self.nnz:
            raise ValueError(f"values must be a 1-D array of nnz = {self.nnz} entries")
        if _dtype_code(data) != self.dtype:
            raise ValueError("values must have the matrix's element type")
        _order_torch(data)
        p, mem, _, keep = _ptr_mem(data)
        _check(self.ctx, load_library().skr_matrix_update_values(self.handle, _VP(p), mem))
        self.version += 1

    def ilu0(self):
        """skr_matrix_ilu0: attach right no-fill ILU factors (used by solves with
        precond='ilu0' until the values change)."""
        _check(self.ctx, load_library().skr_matrix_ilu0(self.ctx.handle, self.handle))
        return self

    @property
    def sell_padding(self) -> float:
        return load_library().skr_matrix_sell_padding(self.handle)

    def close(self):
        if getattr(self, "handle", None):
            load_library().skr_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


@dataclass
class SolveInfo:
    status: int
    iterations: int
    matvecs: int
    outer_iterations: int
    breakdown_iter: int
    rel_res_recursive: float
    rel_res_true: float
    history: np.ndarray = field(repr=False)
    fp64_outer_iterations: int = 0
    single_workgroup: bool = False

    @property
    def status_name(self):
        return STATUS_NAMES.get(self.status, str(self.status))


def opts_default() -> skr_opts:
    o = skr_opts()
    load_library().skr_opts_default(ctypes.byref(o))
    return o


def solve(ctx: Context, A: Matrix, B, method: str, X=None, x0_zero: bool = False, tol: float = 1e-8,
          maxit: int = 10000,
          precision: str = "fp64", inner_tol: float = 1e-4, max_outer: int = 10, preprocess_qr: bool = True,
          check_every: int = 16, use_graph: bool = True, adjoint: bool = False, history_cap: int | None = None,
          precond: str | None = None, fused_small: bool = True):
    """skr_solve.  B: n x s (numpy or torch CUDA tensor).  X: optional initial
    guess / output array of the same kind (a new one is created if None);
    with x0_zero the contents of X are ignored (X0 = 0).  precond='ilu0':
    right ILU(0) preconditioning (A.ilu0() first).  fused_small=False keeps
    small Gl-BiCG / eGl-BiCG / Gl-BiCGStab systems on the general multi-kernel
    schedule.
    Returns (X, SolveInfo)."""
    lib = load_library()
    _check_block(B, A.n, A.dtype, "B")
    if X is not None:
        _check_block(X, A.n, A.dtype, "X", like=B)
    pB, memB, dt, keepB = _ptr_mem(B)
    n, s = B.shape
    if X is None:
        zero_x0 = 1
        if _is_torch(B):
            import torch
            X = torch.zeros_like(B)
        else:
            X = np.zeros_like(keepB)
    else:
        zero_x0 = 1 if x0_zero else 0
        if not _is_torch(X):
            X = np.ascontiguousarray(X, dtype=keepB.dtype)
    pX, memX, _, _ = _ptr_mem(X)
    if memX != memB:
        raise ValueError("B and X must live in the same memory")
    _order_torch(B, X)
    o = opts_default()
    o.tol = tol
    o.maxit = maxit
    o.precision = PRECISIONS[precision]
    o.inner_tol = inner_tol
    o.max_outer = max_outer
    o.preprocess_qr = int(preprocess_qr)
    o.zero_x0 = zero_x0
    o.check_every = check_every
    o.use_graph = int(use_graph)
    o.precond = PRECONDS[precond]
    o.fused_small = int(fused_small)
    cap = history_cap if history_cap is not None else maxit + 2
    hist = np.zeros(max(cap, 1), dtype=np.float64)
    r = skr_result()
    r.history = hist.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    r.history_cap = cap
    rc = lib.skr_solve(ctx.handle, A.handle, s, _VP(pB), s, _VP(pX), s, memB, METHODS[method], ctypes.byref(o),
                       int(adjoint), ctypes.byref(r))
    _check(ctx, rc)
    info = SolveInfo(r.status, r.iterations, r.matvecs, r.outer_iterations, r.breakdown_iter, r.rel_res_recursive,
                     r.rel_res_true, hist[: r.history_len].copy(), r.fp64_outer_iterations,
                     bool(r.single_workgroup))
    return X, info


def spmm(ctx: Context, A: Matrix, X, Y=None, adjoint: bool = False, sync: bool = True):
    """skr_spmm: Y = A X (or A^H X).  With device tensors and sync=False the
    product is only enqueued on the context's stream (the caller orders it)."""
    _check_block(X, A.n, A.dtype, "X")
    if Y is not None:
        _check_block(Y, A.n, A.dtype, "Y", like=X)
    pX, mem, dt, keep = _ptr_mem(X)
    n, s = X.shape
    if Y is None:
        if _is_torch(X):
            import torch
            Y = torch.empty_like(X)
        else:
            Y = np.empty_like(keep)
    pY, memY, _, _ = _ptr_mem(Y)
    if memY != mem:
        raise ValueError("X and Y must live in the same memory")
    if sync:
        _order_torch(X, Y)
    _check(ctx, load_library().skr_spmm(ctx.handle, A.handle, s, _VP(pX), s, _VP(pY), s, mem, int(adjoint)))
    if sync and mem == SKR_MEM_DEVICE:
        import torch
        torch.cuda.synchronize()
    return Y


def precond_apply(ctx: Context, A: Matrix, Z, Y=None, adjoint: bool = False):
    """skr_precond_apply: Y = M^-1 Z (or M^-H Z) with A's ILU(0) factors."""
    _check_block(Z, A.n, A.dtype, "Z")
    if Y is not None:
        _check_block(Y, A.n, A.dtype, "Y", like=Z)
    pZ, mem, dt, keep = _ptr_mem(Z)
    n, s = Z.shape
    if Y is None:
        if _is_torch(Z):
            import torch
            Y = torch.empty_like(Z)
        else:
            Y = np.empty_like(keep)
    pY, memY, _, _ = _ptr_mem(Y)
    if memY != mem:
        raise ValueError("Z and Y must live in the same memory")
    _order_torch(Z, Y)
    _check(ctx, load_library().skr_precond_apply(ctx.handle, A.handle, s, _VP(pZ), s, _VP(pY), s, mem,
                                                 int(adjoint)))
    return Y


def sddmm(ctx: Context, A: Matrix, G, X, scale: float = -1.0, out=None):
    """skr_sddmm: out[k] = scale * sum_c G[i_k, c] conj(X[j_k, c]) on A's pattern."""
    _check_block(G, A.n, A.dtype, "G")
    _check_block(X, A.n, A.dtype, "X", like=G)
    if out is not None and (len(out.shape) != 1 or int(out.shape[0]) != A.nnz or _dtype_code(out) != A.dtype):
        raise ValueError(f"out must be a 1-D array of nnz = {A.nnz} entries of the matrix's element type")
    pG, mem, dt, kg = _ptr_mem(G)
    pX, _, _, kx = _ptr_mem(X)
    n, s = G.shape
    if out is None:
        if _is_torch(G):
            import torch
            out = torch.empty(A.nnz, dtype=G.dtype, device=G.device)
        else:
            out = np.empty(A.nnz, dtype=kg.dtype)
    pO, memO, _, _ = _ptr_mem(out)
    if _ptr_mem(X)[1] != mem or memO != mem:
        raise ValueError("G, X and out must live in the same memory")
    _order_torch(G, X, out)
    _check(ctx, load_library().skr_sddmm(ctx.handle, A.handle, s, _VP(pG), _VP(pX), _VP(pO), scale, mem))
    if mem == SKR_MEM_DEVICE:
        import torch
        torch.cuda.synchronize()
    return out


def block_qr(ctx: Context, Z):
    """skr_block_qr: Z = Q C (CholeskyQR2 on the device).  Returns (Q, C, status)."""
    pZ, mem, dt, kz = _ptr_mem(Z)
    n, s = Z.shape
    if _is_torch(Z):
        import torch
        Q = torch.empty_like(Z)
    else:
        Q = np.empty_like(kz)
    pQ, _, _, _ = _ptr_mem(Q)
    _order_torch(Z, Q)
    C = np.zeros(s * s * (2 if dt == SKR_C64 else 1), dtype=np.float64)
    rc = load_library().skr_block_qr(ctx.handle, n, s, dt, _VP(pZ), _VP(pQ),
                                     C.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), mem)
    _check(ctx, rc)
    Cm = C.view(np.complex128).reshape(s, s) if dt == SKR_C64 else C.reshape(s, s)
    return Q, Cm, rc


def block_qr_noalloc(ctx: Context, Z, Q):
    """skr_block_qr_noalloc: Z = Q C with no device allocation in the library.
    Z and Q: contiguous n x s float64 / complex128 CUDA tensors (s <= 16; Q
    may be Z).  Returns (C, status)."""
    if not (_is_torch(Z) and Z.is_cuda and _is_torch(Q) and Q.is_cuda):
        raise ValueError("Z and Q must be CUDA tensors")
    if len(Z.shape) != 2 or tuple(Q.shape) != tuple(Z.shape) or _dtype_code(Q) != _dtype_code(Z):
        raise ValueError("Q must have Z's shape and element type")
    pZ, _, dt, _ = _ptr_mem(Z)
    pQ, _, _, _ = _ptr_mem(Q)
    n, s = Z.shape
    _order_torch(Z, Q)
    C = np.zeros(s * s * (2 if dt == SKR_C64 else 1), dtype=np.float64)
    rc = load_library().skr_block_qr_noalloc(ctx.handle, n, s, dt, _VP(pZ), _VP(pQ),
                                             C.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(ctx, rc)
    Cm = C.view(np.complex128).reshape(s, s) if dt == SKR_C64 else C.reshape(s, s)
    return Cm, rc
