"""MI355X (gfx950) simultaneous short-recurrence Krylov solvers.

Solves A X = B for a sparse non-Hermitian A and a block of s right-hand sides
with the global, economic-global and QR-stabilised block variants of BiCG, QMR
and BiCGStab of Rashedi, Birk, Frommer and Ebadi (arXiv 1504.04395).  All
arithmetic runs in the HIP library ``libskrylov.so`` behind the C ABI of
``include/skrylov.h``; this package is its ctypes binding.
"""
from ._binding import (  # noqa: F401
    LIB_PATH, METHODS, PRECISIONS, PRECONDS, STATUS_NAMES, Context, Matrix, SkrError, SolveInfo, block_qr,
    block_qr_noalloc,
    load_library, opts_default, precond_apply, sddmm, solve, spmm,
)


def __getattr__(name):
    # the autograd wrapper imports torch; load it on first use only
    if name in ("SparseSolve", "sparse_solve"):
        from . import autograd
        return getattr(autograd, name)
    raise AttributeError(name)
