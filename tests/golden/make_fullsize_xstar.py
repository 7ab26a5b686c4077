"""Write sampled rows of X* = A^{-1} B for the benchmark workload.

The workload is the 3D convection-diffusion problem on a 128^3 grid
(beta = (30, 20, 10)) with 16 Gaussian right-hand sides (seed 0).  X* is the
oracle's eGl-QMR solution (Section 4) run to a relative residual of 1e-12,
the best FP64 solution the oracle offers; it calls only ``oracle/`` and
``inputs/``.  The file holds the rows that numpy's default_rng(11) draws
(256 of them, plus the first and the last row), one per line: the row index
and its 16 values to 17 significant digits.  The GPU tests compare the
mixed-precision solution with these rows.

    python tests/golden/make_fullsize_xstar.py
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import inputs as I  # noqa: E402
import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "fullsize_xstar_rows.txt")


def sample_rows(n: int) -> np.ndarray:
    rng = np.random.default_rng(11)
    return np.unique(np.concatenate([rng.choice(n, 256, replace=False), [0, n - 1]]))


def main() -> None:
    A = I.convdiff3d(128, (30.0, 20.0, 10.0))
    B = I.gaussian_block(A.n, 16, seed=0)
    t = time.time()
    r = O.solve(A, B, "egl_qmr", tol=1e-12, maxit=5000)
    rows = sample_rows(A.n)
    with open(OUT, "w") as f:
        f.write("# X* = A^{-1} B on the 128^3 convection-diffusion workload (beta = (30, 20, 10), 16 Gaussian\n"
                "# right-hand sides, seed 0): the oracle's eGl-QMR run to a relative residual of 1e-12\n"
                f"# (status {r.status}, {r.iterations} iterations, true relative residual {r.rel_res_true:.3e},\n"
                f"# ||X*||_F = {np.linalg.norm(r.X):.17e}).  Rows drawn by numpy default_rng(11).\n"
                "# Written by make_fullsize_xstar.py, which calls only oracle/ and inputs/.\n"
                "# row  X*[row, 0..15]\n")
        for i in rows:
            f.write(f"{i} " + " ".join(f"{v:.17e}" for v in r.X[i]) + "\n")
    print(f"status {r.status} it {r.iterations} res {r.rel_res_true:.3e} ({time.time() - t:.0f} s) -> {OUT}")


if __name__ == "__main__":
    main()
