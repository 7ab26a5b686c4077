"""CPU test of the library's SELL-C-sigma build (host code in csrc/sell.hpp),
through a small g++ harness (tests/host/sell_host_main.cpp); no GPU involved.

Checked against the definition of the format: rows stably sorted by length,
longest first, inside windows of sigma rows; chunks of C sorted positions,
column-major, padded to their longest row; every nonzero in exactly one slot
with its column and CSR position; padding slots point at their row's own
column with CSR position -1."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1504_04395_amd", "csrc")


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    out = str(tmp_path_factory.mktemp("sell") / "sell_host")
    subprocess.run([gxx, "-O2", "-std=c++17", f"-I{CSRC}", os.path.join(HERE, "host", "sell_host_main.cpp"),
                    "-o", out], check=True, capture_output=True, timeout=300)
    return out


def _pattern(n, seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 12, size=n)
    if n > 4:
        lens[rng.choice(n, size=max(1, n // 30), replace=False)] = 0
        lens[rng.choice(n, size=2, replace=False)] = 60
    lens = np.minimum(lens, n)               # distinct columns per row
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    ci = np.concatenate([np.sort(rng.choice(n, size=int(L), replace=False)) for L in lens] or [[]])
    return rp, ci.astype(np.int64)


def _build(harness, tmp_path, n, rp, ci, C, sigma):
    f = tmp_path / "p.txt"
    with open(f, "w") as fh:
        fh.write(f"{n} {len(ci)} {C} {sigma}\n")
        fh.write(" ".join(map(str, rp)) + "\n")
        fh.write(" ".join(map(str, ci)) + "\n")
    out = subprocess.run([harness, str(f)], check=True, capture_output=True, text=True, timeout=120).stdout
    lines = out.splitlines()
    assert lines[0] == "ok", lines[0]
    arr = [np.array(l.split(), dtype=np.int64) for l in lines[1:6]]
    return dict(zip(("cptr", "clen", "row", "ci", "idx"), arr))


@pytest.mark.parametrize("C,sigma", [(16, 16), (16, 256), (32, 32), (32, 128), (64, 64), (64, 8192)])
@pytest.mark.parametrize("n", [1, 15, 16, 17, 1000 + 37])
def test_sell_layout_matches_its_definition(harness, tmp_path, n, C, sigma):
    rp, ci = _pattern(n, seed=n + C + sigma)
    h = _build(harness, tmp_path, n, rp, ci, C, sigma)
    lens = np.diff(rp)
    # sorted positions: a stable sort by descending length inside each window
    order = np.concatenate([w0 + np.argsort(-lens[w0:w0 + sigma], kind="stable") for w0 in range(0, n, sigma)])
    assert np.array_equal(h["row"], order)
    nch = (n + C - 1) // C
    sl = np.concatenate([lens[order], np.zeros(nch * C - n, dtype=lens.dtype)])
    clen = sl.reshape(nch, C).max(axis=1)
    assert np.array_equal(h["clen"], clen)
    assert np.array_equal(h["cptr"], np.concatenate([[0], np.cumsum(clen * C)]))
    seen = np.zeros(len(ci), dtype=np.int64)
    for ch in range(nch):
        for r in range(C):
            p = ch * C + r
            i = order[p] if p < n else 0
            L = lens[i] if p < n else 0
            e = h["cptr"][ch] + np.arange(clen[ch]) * C + r
            real = np.arange(clen[ch]) < L
            assert np.array_equal(h["idx"][e[real]], rp[i] + np.arange(L))
            assert np.array_equal(h["ci"][e[real]], ci[rp[i]:rp[i] + L])
            assert np.all(h["idx"][e[~real]] == -1) and np.all(h["ci"][e[~real]] == i)
            seen[rp[i]:rp[i] + L] += 1 if p < n else 0
    assert np.all(seen == 1)                 # every nonzero in exactly one slot


def test_sell_empty_pattern(harness, tmp_path):
    n = 40
    h = _build(harness, tmp_path, n, np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int64), 16, 16)
    assert np.all(h["clen"] == 0) and h["cptr"][-1] == 0 and len(h["ci"]) == 0
