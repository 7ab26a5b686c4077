"""CPU-only checks of the boundary: the built library loads and exports every
function include/skrylov.h declares; the binding refuses bad input before any
device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skrylov.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(skr_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("skr_solve", "skr_spmm", "skr_sddmm", "skr_matrix_create", "skr_context_create", "skr_block_qr"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1504_04395_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(pkg.LIB_PATH)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_signatures_cover_header():
    from paper_1504_04395_amd import _binding
    assert set(_declared()) == set(_binding._SIGS)


def test_missing_library_fails_loudly(tmp_path):
    from paper_1504_04395_amd import _binding
    saved = _binding._lib
    _binding._lib = None
    try:
        with pytest.raises(RuntimeError, match="not built"):
            _binding.load_library(str(tmp_path / "nope.so"))
    finally:
        _binding._lib = saved


def test_oracle_and_gpu_path_are_independent():
    """The oracle imports nothing from the GPU package and vice versa."""
    for d, banned in (("oracle", "paper_1504_04395_amd"), ("paper_1504_04395_amd", "oracle")):
        for f in os.listdir(os.path.join(ROOT, d)):
            if f.endswith(".py"):
                src = open(os.path.join(ROOT, d, f)).read()
                assert not re.search(rf"^\s*(from|import)\s+{banned}\b", src, flags=re.M), (d, f)


def test_opts_default_without_gpu():
    import paper_1504_04395_amd as pkg
    if not os.path.exists(pkg.LIB_PATH):
        pytest.skip("library not built")
    o = pkg.opts_default()
    assert o.tol == 1e-8 and o.maxit == 10000 and o.preprocess_qr == 1 and o.zero_x0 == 1
