"""Host-side behaviour of bench.py (no GPU): the one-GPU guard and the
hardware-counter record it reports as roofline.traffic."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_counter_record_matches_the_spmm_source():
    t = bench.counter_traffic("k_spmm_csr8<double,EpiNone>")
    assert isinstance(t, int) and t > 720_240_644     # at least the algorithmic bytes
    assert bench.counter_traffic("some_other_kernel") is None


def test_counter_record_is_dropped_when_the_source_changes(monkeypatch, tmp_path):
    # a copy of the tree's layout whose spmm.hpp differs from the one the counters were taken on
    (tmp_path / "profiles").mkdir()
    (tmp_path / "paper_1504_04395_amd" / "csrc").mkdir(parents=True)
    src = os.path.join(ROOT, "profiles", "spmm_csr_convdiff3d128_s16_counters.md")
    (tmp_path / "profiles" / "spmm_csr_convdiff3d128_s16_counters.md").write_text(open(src).read())
    spmm = open(os.path.join(ROOT, "paper_1504_04395_amd", "csrc", "spmm.hpp")).read()
    (tmp_path / "paper_1504_04395_amd" / "csrc" / "spmm.hpp").write_text(spmm + "\n// changed\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.counter_traffic("k_spmm_csr8<double,EpiNone>") is None
