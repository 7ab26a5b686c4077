"""Write the oracle's iteration counts on the benchmark workload.

The workload is the 128^3 convection-diffusion problem with 16 Gaussian
right-hand sides (FP64, tol 1e-8, at most 1200 iterations), solved by
Bl-BiCG-rQ (Algorithm 5), eGl-QMR (Section 4) and Bl-BiCGStab-rQ (closing
paragraph of Section 4).  Only ``oracle/`` and ``inputs/`` are called.

Seed 0 is the run on the workload's own inputs; seed k > 0 perturbs B by
1e-15 relative noise drawn from numpy's default_rng(k).  Their counts are the oracle's own spread: a Krylov recurrence
amplifies rounding differences, so two correct FP64 implementations of the
same method stop at counts that differ by about this much.

Output: one line per run, appended to ``fullsize_iterations.txt`` next to this
script (``--grid`` selects a smaller cube of the same family).

    python tests/golden/make_fullsize_counts.py --method bl_bicg_rq --seeds 0
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import inputs as I  # noqa: E402
import oracle as O  # noqa: E402

OUT = os.path.join(HERE, "fullsize_iterations.txt")
HEADER = ("# Oracle iteration counts, 3D convection-diffusion (beta = (30, 20, 10)), 16 Gaussian right-hand sides\n"
          "# (seed 0), FP64, tol 1e-8 on the recursive residual, at most 1200 iterations.  seed 0 = the inputs\n"
          "# themselves; seed k > 0 = B * (1 + 1e-15 * N(0,1)) from numpy default_rng(k).  Written by\n"
          "# make_fullsize_counts.py, which calls only oracle/ and inputs/.\n"
          "# grid  method          seed  status  iterations  rel_res_true\n")


def perturbed(B: np.ndarray, seed: int) -> np.ndarray:
    if seed == 0:
        return B
    rng = np.random.default_rng(seed)
    return B * (1 + 1e-15 * rng.standard_normal(B.shape))


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--method", required=True, choices=["bl_bicg_rq", "egl_qmr", "bl_bicgstab_rq"])
    ap.add_argument("--grid", type=int, default=128)
    ap.add_argument("--seeds", type=int, nargs="+", default=[0], help="0 = unperturbed; k > 0 = perturbed")
    ap.add_argument("--out", default=OUT)
    a = ap.parse_args()
    A = I.convdiff3d(a.grid, (30.0, 20.0, 10.0))
    B = I.gaussian_block(A.n, 16, seed=0)
    for seed in a.seeds:
        t = time.time()
        r = O.solve(A, perturbed(B, seed), a.method, tol=1e-8, maxit=1200)
        line = f"{a.grid:<5d} {a.method:<15s} {seed:<5d} {r.status:<7d} {r.iterations:<11d} {r.rel_res_true:.3e}\n"
        new = not os.path.exists(a.out)
        with open(a.out, "a") as f:
            if new:
                f.write(HEADER)
            f.write(line)
        print(line.strip(), f"({time.time() - t:.0f} s)", flush=True)


if __name__ == "__main__":
    main()
