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


def _record_sha():
    import hashlib
    text = open(os.path.join(ROOT, "profiles", "spmm_csr_convdiff3d128_s16_counters.md")).read()
    rec = [l for l in text.splitlines() if l.startswith("- `spmm.hpp sha256`") or l.startswith("- spmm.hpp sha256")]
    cur = hashlib.sha256(open(os.path.join(ROOT, "paper_1504_04395_amd", "csrc", "spmm.hpp"), "rb").read())
    return rec, cur.hexdigest()


def test_counter_record_matches_the_spmm_source():
    """The traffic figure is reported exactly while the counters' record names
    the current source (then it is at least the algorithmic bytes)."""
    rec, cur = _record_sha()
    t = bench.counter_traffic("k_spmm_csr8<double,EpiNone>")
    if rec and cur in rec[0]:
        assert isinstance(t, int) and t > 720_240_644     # at least the algorithmic bytes
    else:
        assert t is None
    assert bench.counter_traffic("some_other_kernel") is None


def test_oracle_counts_file(tmp_path):
    f = tmp_path / "counts.txt"
    f.write_text("# grid method seed status iterations res\n"
                 "128   bl_bicg_rq      0     0       483         9.1e-09\n"
                 "128   bl_bicg_rq      1     0       470         9.0e-09\n"
                 "128   egl_qmr         0     0       433         9.9e-09\n"
                 "64    egl_qmr         0     0       200         9.9e-09\n"
                 "128   bl_bicgstab_rq  0     1       1200        1.0e-03\n")
    assert bench.oracle_counts(128, str(f)) == {"bl_bicg_rq": 483, "egl_qmr": 433}
    assert bench.oracle_counts(64, str(f)) == {"egl_qmr": 200}
    assert bench.oracle_counts(128, str(tmp_path / "missing.txt")) == {}
    assert isinstance(bench.host_cpu_model(), str)


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
