"""CPU model of the launch geometry shared by the streaming kernels
(csrc/engine.hpp `make_env`, csrc/common.hpp `xcd_chunk`, the row and tile
loops of csrc/blk.hpp and csrc/glk.hpp).

For ragged n and every block width it checks that

  - `xcd_chunk` maps the workgroups one-to-one onto the row chunks;
  - the chunks, the 16-row tiles each wave sweeps, the lane-group row passes
    and the flat element loop cover every row (element) exactly once;
  - at the largest n the matrix set-up accepts, no int32 row index formed by
    these loops (a chunk end, a pass start one stride past the end, the 8-lane
    SpMM's next-pass prefetch) overflows.

The model restates the launch arithmetic; a change to one side must be made on
the other.
"""
import numpy as np
import pytest

BLOCK = 256
WAVES = BLOCK // 64
MAX_ROWS = (1 << 31) - (1 << 20)      # the largest n skr_matrix_create accepts
INT32_MAX = (1 << 31) - 1


def env(n, s):
    nb = (n + 63) // 64
    nb = ((nb + 7) // 8) * 8
    nb = max(8, min(2048, nb))
    rpc = (n + nb - 1) // nb
    rpc = ((rpc + 15) // 16) * 16
    total = n * s
    per = (total + nb - 1) // nb
    per = ((per + BLOCK - 1) // BLOCK) * BLOCK
    L = min(16, 1 << (s.bit_length() - 1))
    return nb, rpc, per, total, L


def xcd_chunk(b, nb):
    return (b & 7) * (nb >> 3) + (b >> 3)


@pytest.mark.parametrize("nb", [8, 16, 24, 512, 2048])
def test_xcd_chunk_is_a_bijection(nb):
    assert sorted(xcd_chunk(b, nb) for b in range(nb)) == list(range(nb))


@pytest.mark.parametrize("n", [1, 15, 16, 17, 63, 64, 65, 1000, 4099, 131_072 + 5])
@pytest.mark.parametrize("s", [1, 3, 16, 17, 32])
def test_row_tile_and_flat_loops_cover_once(n, s):
    nb, rpc, per, total, L = env(n, s)
    assert rpc % 16 == 0 and nb % 8 == 0
    tiles = np.zeros(n, dtype=np.int64)     # 16-row tiles swept by the waves (blk.hpp kernels)
    passes = np.zeros(n, dtype=np.int64)    # SKR_ROW_LOOP lane-group passes (glk.hpp kernels)
    flat = np.zeros(total, dtype=np.int64)  # SKR_FLAT_LOOP
    rpb = BLOCK // L
    for b in range(nb):
        c = xcd_chunk(b, nb)
        r0 = c * rpc
        r1 = min(n, r0 + rpc)
        for w in range(WAVES):
            for t0 in range(r0 + 16 * w, r1, 16 * WAVES):
                rows = t0 + np.arange(16)
                tiles[rows[rows < r1]] += 1
        for base in range(r0, r1, rpb):
            rows = base + np.arange(rpb)
            passes[rows[rows < r1]] += 1
        e0 = c * per
        e1 = min(e0 + per, total)
        if e0 < e1:
            flat[e0:e1] += 1
    assert np.all(tiles == 1) and np.all(passes == 1) and np.all(flat == 1)


@pytest.mark.parametrize("s", [1, 2, 16, 32])
def test_no_int32_overflow_at_the_row_limit(s):
    n = MAX_ROWS
    nb, rpc, per, total, L = env(n, s)
    # chunk ends and the first pass start past a chunk end
    last_chunk_end = (nb - 1) * rpc + rpc
    assert last_chunk_end + 16 * WAVES <= INT32_MAX
    assert last_chunk_end + BLOCK <= INT32_MAX
    # the 8-lane SpMM: rows per XCD, and the next-pass prefetch one stride past the last pass
    per_xcd = ((n + 7) // 8 + 63) // 64 * 64
    step = (nb >> 3) * 64
    assert 8 * per_xcd + step + 64 <= INT32_MAX
    assert n + step + 64 <= INT32_MAX
    # the SELL kernel: chunk starts of the last workgroups (past the last chunk) times C
    for C in (16, 32, 64):
        nchunks = (n + C - 1) // C
        cpb = (nchunks + nb - 1) // nb
        assert ((nb - 1) * cpb + cpb) * C + BLOCK <= INT32_MAX


def _sell_layout(lens, C, sigma):
    """Chunk widths and offsets of SELL-C-sigma by its definition (rows sorted by
    length, longest first, inside windows of sigma rows; chunks of C sorted
    positions padded to their longest row)."""
    n = lens.size
    order = np.concatenate([w0 + np.argsort(-lens[w0:w0 + sigma], kind="stable") for w0 in range(0, n, sigma)])
    nch = (n + C - 1) // C
    clen = np.array([lens[order[c * C:(c + 1) * C]].max(initial=0) for c in range(nch)], dtype=np.int64)
    cptr = np.concatenate([[0], np.cumsum(clen * C)])
    return clen, cptr


def walk_sell16(n, lens, C, sigma, nb):
    """Model of k_spmm_sell16's walk: workgroup b owns chunks [xcd_chunk(b) * cpb,
    +cpb); rounds (chunk, pass r0, slot k) advance by 8 slots, then by 16 sorted
    positions, then to the next chunk; chunks of width 0 only write zeros.  Lane
    lw < 32 of wave w loads slot k + lw // 4 of position r0 + 4 w + lw % 4.
    Returns (writes per sorted position, loads per stored slot, max load index)."""
    U = 8
    clen, cptr = _sell_layout(lens, C, sigma)
    slots = int(cptr[-1])
    nchunks = clen.size
    cpb = (nchunks + nb - 1) // nb
    writes = np.zeros(n, dtype=np.int64)
    loads = np.zeros(max(slots, 1), dtype=np.int64)
    lw = np.arange(32)
    for b in range(nb):
        cb = xcd_chunk(b, nb) * cpb
        ce = min(nchunks, cb + cpb)
        for ch in range(cb, ce):
            width, e0 = int(clen[ch]), int(cptr[ch])
            for r0 in range(0, C, 16):
                for w in range(4):
                    pos = ch * C + r0 + 4 * w + np.arange(4)
                    writes[pos[pos < n]] += 1
                    for k in range(0, width, U):                   # no rounds in a width-0 chunk
                        kk = k + (lw >> 2)
                        ok = kk < width
                        e = np.where(ok, e0 + kk * C + r0 + 4 * w + (lw & 3), 0)
                        assert np.all((e >= 0) & (e < max(slots, 1)))
                        assert np.all((lw >> 2) < U) and np.all((lw & 3) < 4)   # LDS [8][4] per wave
                        np.add.at(loads, e[ok], 1)
    return writes, loads, slots


@pytest.mark.parametrize("n", [1, 17, 1000, 20_000 + 9])
@pytest.mark.parametrize("C", [16, 32, 64])
@pytest.mark.parametrize("sigma_mult", [1, 16])
def test_sell16_walk_writes_every_position_once_and_loads_every_slot_once(n, C, sigma_mult):
    """k_spmm_sell16 on ragged rows (empty rows, long rows, a partial last chunk,
    chunks of empty rows): every sorted position is written once and every
    stored slot (padding included) is loaded exactly once, all in bounds."""
    rng = np.random.default_rng(n + C)
    lens = rng.integers(0, 12, size=n)
    lens[rng.random(n) < 0.2] = 0
    if n > 40:
        lens[rng.choice(n, 3, replace=False)] = 37
        lens[: 2 * C] = 0                                   # whole chunks of empty rows
    nb = env(n, 1)[0]
    writes, loads, slots = walk_sell16(n, lens, C, C * sigma_mult, nb)
    assert np.all(writes == 1)
    if slots:
        assert np.all(loads == 1)


def test_sell16_all_empty_matrix():
    n, C = 100, 16
    writes, loads, slots = walk_sell16(n, np.zeros(n, dtype=np.int64), C, 256, env(n, 1)[0])
    assert slots == 0 and np.all(writes == 1)


def _per_xcd_sweep(n, nb, per_xcd, rows_per_pass, row_of):
    """Rows touched by a per-XCD sweep: XCD b & 7 owns rows [xcd * per_xcd, +per_xcd),
    its workgroup q starts at q * rows_per_pass and strides by nq * rows_per_pass;
    row_of(base) gives the rows one pass covers."""
    seen = np.zeros(n, dtype=np.int64)
    nq = nb >> 3
    for b in range(nb):
        xcd, q = b & 7, b >> 3
        r0 = xcd * per_xcd
        r1 = min(n, r0 + per_xcd)
        for base in range(r0 + q * rows_per_pass, r1, nq * rows_per_pass):
            rows = row_of(base)
            np.add.at(seen, rows[rows < r1], 1)
    return seen


@pytest.mark.parametrize("n", [1, 33, 1000, 20_000 + 11])
def test_sixteen_lane_csr_and_single_vector_sweeps_cover_once(n):
    nb, _, _, _, _ = env(n, 16)
    # k_spmm_csr: 16 lanes per row, RP row passes of 16 lane groups (16 rows) per pass
    per_xcd = ((n + 7) // 8 + 31) // 32 * 32
    for RP in (1, 2):
        seen = _per_xcd_sweep(n, nb, per_xcd, RP * 16,
                              lambda base: (base + 16 * np.arange(RP)[:, None] + np.arange(16)[None, :]).ravel())
        assert np.all(seen == 1), RP
    # k_spmv_csr: 8 lanes per row, 32 rows per pass
    seen = _per_xcd_sweep(n, nb, per_xcd, 32, lambda base: base + np.arange(32))
    assert np.all(seen == 1)
