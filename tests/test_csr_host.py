"""CPU test of the library's CSR set-up (host code in csrc/csr_host.hpp)
through a small g++ harness (tests/host/csr_host_main.cpp); no GPU involved.

Validation: each malformed input is rejected with its reason.  A^H pattern:
equal to scipy's transpose, rows in increasing column order, and perm maps
every A^H entry to the A entry with the transposed indices."""
import os
import shutil
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1504_04395_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("csr") / "csr_host")
    subprocess.run([gxx, "-O2", "-std=c++17", f"-I{CSRC}", os.path.join(HERE, "host", "csr_host_main.cpp"),
                    "-o", out], check=True, capture_output=True, timeout=300)
    return out


def _run(harness, tmp_path, n, rp, ci):
    f = tmp_path / "c.txt"
    with open(f, "w") as fh:
        fh.write(f"{n} {len(ci)}\n" + " ".join(map(str, rp)) + "\n" + " ".join(map(str, ci)) + "\n")
    return subprocess.run([harness, str(f)], check=True, capture_output=True, text=True, timeout=120).stdout


@pytest.mark.parametrize("n,density,seed", [(1, 1.0, 0), (7, 0.4, 1), (300, 0.02, 2), (2000, 0.003, 3)])
def test_adjoint_pattern_is_the_transpose(harness, tmp_path, n, density, seed):
    M = sp.random(n, n, density=density, format="csr", random_state=seed)
    M.sort_indices()
    out = _run(harness, tmp_path, n, M.indptr, M.indices).splitlines()
    assert out[0] == "ok"
    rpH, ciH, perm = (np.array(l.split(), dtype=np.int64) for l in out[1:4])
    T = sp.csr_array(M.T)
    T.sort_indices()
    assert np.array_equal(rpH, T.indptr) and np.array_equal(ciH, T.indices)
    rows_A = np.repeat(np.arange(n), np.diff(M.indptr))
    rows_H = np.repeat(np.arange(n), np.diff(rpH))
    assert np.array_equal(np.sort(perm), np.arange(M.nnz))          # a permutation
    assert np.array_equal(M.indices[perm], rows_H)                   # A^H[j, i] comes from A[i, j]
    assert np.array_equal(rows_A[perm], ciH)


def test_empty_pattern(harness, tmp_path):
    out = _run(harness, tmp_path, 5, [0] * 6, []).splitlines()
    assert out[0] == "ok" and out[1].split() == ["0"] * 6


@pytest.mark.parametrize("rp,ci,why", [
    ([1, 1, 2], [0, 1], "row_ptr[0] must be 0"),
    ([0, 1, 1], [0, 1], "row_ptr[0] must be 0 and row_ptr[n] = nnz"),
    ([0, 2, 1, 3], [0, 1, 2], "non-decreasing"),
    ([0, 1, 2], [0, 2], "out of range"),
    ([0, 1, 2], [0, -1], "out of range"),
    ([0, 2, 2], [1, 0], "strictly increasing"),
    ([0, 2, 2], [1, 1], "strictly increasing"),
])
def test_malformed_csr_is_rejected(harness, tmp_path, rp, ci, why):
    n = len(rp) - 1
    out = _run(harness, tmp_path, n, rp, ci).strip()
    assert out.startswith("ERROR") and why in out, out
