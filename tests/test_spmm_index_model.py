"""CPU model of the launch geometry and per-lane indexing of the 8-lane CSR
sparse x block kernel (`k_spmm_csr8` in csrc/spmm.hpp, launched from
csrc/engine.hpp).  It walks every workgroup and pass of the grid the engine
launches and checks, for ragged sizes, that

  - every (row, column) of Y is written exactly once;
  - every row-pointer read (this pass and the prefetched next pass) is inside
    rp[0..n];
  - every entry read (first U entries, the prefetched next-pass entries, and the
    in-place reads of longer rows) is inside ci/va, which hold max(nnz, 1)
    entries;
  - every epilogue operand read (tile layout for the Grams, the lane's own rows
    and columns for the row sums) is inside the n x s block;
  - the LDS staging of a round's entries: each lane of a wave writes one slot
    of the wave's [16 rows][8 slots] area, every slot is written exactly once,
    and the 8 slots a lane reads back for its row are the ones the 8 lanes of
    that row wrote.

The model restates the kernel's index arithmetic; a change to one side must be
made on the other.
"""
import numpy as np
import pytest

U = 8          # entries per lane per round
BLOCK = 256    # threads per workgroup


def engine_nb(n):
    nb = (n + 63) // 64
    nb = ((nb + 7) // 8) * 8
    return max(8, min(2048, nb))


def walk_csr8(n, rp, s, nb):
    nnz_alloc = max(int(rp[-1]), 1)
    per_xcd = ((n + 7) // 8 + 63) // 64 * 64
    written = np.zeros((n, s), dtype=np.int64)
    t = np.arange(BLOCK)
    lane = t & 15
    half = lane >> 3
    l8 = lane & 7
    w = t >> 6
    g = (t >> 4) & 3
    tc = t & 15
    tq = (t >> 4) & 3
    colok = 2 * l8 < s
    nq = nb >> 3
    step = nq * 64

    def rows_of(base, r1):
        i = np.stack([base + 16 * w + 8 * p + 2 * g + half for p in range(2)])
        valid = i < r1
        ii = np.minimum(i, n - 1)                                        # loaded for every lane
        assert np.all(ii >= 0) and np.all(ii + 1 <= n)                   # rp[ii], rp[ii + 1]
        k0 = np.where(valid, rp[ii], 0)
        k1 = np.where(valid, rp[ii + 1], 0)
        return i, valid, k0, k1

    def entries(k0, k1, off):
        k = k0 + off + l8
        kc = np.maximum(0, np.minimum(k, k1 - 1))
        assert np.all((kc >= 0) & (kc < nnz_alloc))                       # ci[kc], va[kc]
        return kc

    for b in range(nb):
        xcd, q = b & 7, b >> 3
        r0 = xcd * per_xcd
        r1 = min(n, r0 + per_xcd)
        base = r0 + q * 64
        if base >= r1:
            continue
        i, valid, k0, k1 = rows_of(base, r1)
        entries(k0, k1, 0)
        while base < r1:
            wb = base + 16 * w
            # Gram epilogue operand, tile layout
            for v in range(4):
                r = wb + 4 * v + tq
                ok = (r < r1) & (tc < s)
                row = np.where(ok, r, base)
                col = np.where(ok, tc, 0)
                assert np.all((row >= 0) & (row < n) & (col >= 0) & (col < s))
            # row-sum epilogue operands, the lane's own rows and columns
            for p in range(2):
                ok = valid[p] & colok
                row = np.where(ok, i[p], base)
                assert np.all((row >= 0) & (row < n))
            ni, nvalid, nk0, nk1 = rows_of(base + step, r1)               # next pass's row pointers
            off = 0
            while True:
                lane_more = np.any(k0 + off + U < k1, axis=0)              # either of the lane's rows
                if off == 0:
                    entries(nk0, nk1, 0)                                   # next pass's first entries
                if not np.any(lane_more):
                    break
                # a wave continues while any of its lanes has more (__any); continuing
                # every wave here checks a superset of the kernel's reads
                entries(k0, k1, off + U)
                off += U
            for p in range(2):
                wr = valid[p] & colok
                for c in (0, 1):
                    np.add.at(written, (i[p][wr], 2 * l8[wr] + c), 1)
            i, valid, k0, k1 = ni, nvalid, nk0, nk1
            base += step
    return written


def test_csr8_lds_staging_layout():
    t = np.arange(BLOCK)
    lane = t & 15
    half = lane >> 3
    l8 = lane & 7
    w = t >> 6
    g = (t >> 4) & 3
    waves = BLOCK // 64
    owner = -np.ones((waves, 16, U), dtype=np.int64)
    for p in range(2):
        lr = 8 * p + 2 * g + half
        assert np.all((lr >= 0) & (lr < 16))
        for th in range(BLOCK):
            assert owner[w[th], lr[th], l8[th]] == -1          # written once
            owner[w[th], lr[th], l8[th]] = th
    assert np.all(owner >= 0)                                  # every slot written
    for p in range(2):
        lr = 8 * p + 2 * g + half
        for th in range(BLOCK):
            writers = owner[w[th], lr[th], :]
            # the writers of the row a lane reads are the 8 lanes of its own row
            # group (same wave, same 16-lane group, same half), slot u by lane u
            assert np.all(w[writers] == w[th]) and np.all(g[writers] == g[th]) and np.all(half[writers] == half[th])
            assert np.array_equal(l8[writers], np.arange(U))


def _ragged_rp(n, seed):
    rng = np.random.default_rng(seed)
    lens = rng.integers(0, 10, size=n)
    if n > 4:
        lens[rng.choice(n, size=max(1, n // 40), replace=False)] = 0
        lens[rng.choice(n, size=2, replace=False)] = 37                   # several rounds of U
    return np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)


@pytest.mark.parametrize("n", [1, 7, 63, 64, 65, 1037, 20_000 + 37])
@pytest.mark.parametrize("s", [2, 4, 16])
def test_csr8_covers_every_entry_once_and_stays_in_bounds(n, s):
    rp = _ragged_rp(n, seed=n + s)
    written = walk_csr8(n, rp, s, engine_nb(n))
    assert np.all(written == 1)


def test_csr8_empty_matrix_reads_the_one_allocated_slot():
    n = 300
    rp = np.zeros(n + 1, dtype=np.int64)          # nnz = 0: ci/va hold one zero slot
    written = walk_csr8(n, rp, 16, engine_nb(n))
    assert np.all(written == 1)


@pytest.mark.parametrize("nb", [8, 16, 2048])
def test_csr8_any_grid_width(nb):
    n = 5000 + 3
    written = walk_csr8(n, _ragged_rp(n, seed=3), 16, nb)
    assert np.all(written == 1)
