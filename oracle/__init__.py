"""CPU oracle for the simultaneous short-recurrence Krylov solvers of
Rashedi, Birk, Frommer and Ebadi, "On short recurrence Krylov type methods for
linear systems with many right-hand sides" (arXiv 1504.04395).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
numpy/scipy FP64 implementation of what the GPU path computes.  Only the test
suite, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py``
may import it.  The GPU path (``paper_1504_04395_amd``) never imports it, and
this package imports nothing from the GPU path; the two share only the seeded
input generators in ``inputs/``.

Pins (what fixes each function independently of itself) are the ``-m "not gpu"``
tests under ``tests/test_oracle_*.py``.  Bl-BiCGStab-rQ, which the paper does not
write out (its step order is a reading, see ``krylov.bl_bicgstab_rq``), is pinned
by its s = 1 reduction to scipy's bicgstab, by equality with block BiCGStab
(El Guennouni et al.) over the first iterations, and by its residual equalling
psi_k(A) applied to the block BiCG residual, block BiCG itself being pinned by
brute-force Petrov-Galerkin conditions.  Values the paper prints pin the
methods as well: the iteration counts of Table 2 (Section 5.2, Examples 1-3,
with and without ILU(0)) and the matrix-vector product relations between the
method families of Section 5.3.
"""
from .krylov import (  # noqa: F401
    METHODS, PIN_METHODS, Result, solve, qr_pos, tr,
    STATUS_OK, STATUS_NOT_CONVERGED, STATUS_BREAKDOWN, STATUS_DIVERGED,
)
from .grad import dense_solve_grad, sddmm  # noqa: F401
