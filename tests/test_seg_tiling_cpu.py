"""The device-offset tile and wave tables, stated on the CPU (no GPU).

The segmented device-offset calls build the tile table (tbase) and the wave
table on the GPU in three kernels over rows of 1024 segments
(csrc/segmented.hip: seg_count_kernel, seg_rows_kernel,
seg_finish_kernel). This test restates their integer arithmetic in Python
and checks, on random offsets with empty, short and long segments, that
  * tbase is the exclusive prefix sum of the tiles per segment;
  * the waves' ranges [wt[2w], wt[2w+2]) cover the tiles 0..NT-1 exactly
    once, in order, and each wave's segment is at or before the segment of
    its first tile (the tile walk moves forward from it);
  * the first tile of every wave equals the one the plans' host wave table
    (build_wave_table) gives for the same cost model.
Results do not depend on the partition; this guards against tiles reduced
twice or not at all.
"""
import numpy as np
import pytest

ROW = 1024


def tiles_of(off, ts):
    lens = np.diff(off)
    return np.where(lens > 0, (lens + ts - 1) // ts, 0)


def device_tables(off, ts, c0, nw):
    """The three kernels' arithmetic, row by row."""
    nseg = len(off) - 1
    nrow = (nseg + ROW - 1) // ROW
    tiles = tiles_of(off, ts)
    tbase = np.zeros(nseg + 1, dtype=np.int64)
    rows = np.zeros(nrow + 1, dtype=np.int64)
    for r in range(nrow):  # 1. in-row exclusive scan, row totals
        seg = tiles[r * ROW:(r + 1) * ROW]
        inc = np.cumsum(seg)
        tbase[r * ROW:r * ROW + len(seg)] = inc - seg
        rows[r] = inc[-1]
    carry = 0
    for r in range(nrow):  # 2. rows' exclusive prefix
        v = rows[r]
        rows[r] = carry
        carry += v
    rows[nrow] = carry
    NT = int(carry)
    wt = np.full(2 * (nw + 1), -1, dtype=np.int64)
    C = int(off[nseg] - off[0]) + c0 * NT
    wt[2 * nw] = NT
    wt[2 * nw + 1] = nseg - 1
    if C == 0:
        wt[:2 * nw] = 0
    for sg in range(nseg):  # 3. global bases and wave entries
        tb = int(tbase[sg] + rows[sg // ROW])
        tbase[sg] = tb
        if C == 0:
            continue
        ln = int(off[sg + 1] - off[sg])
        ntl = (ln + ts - 1) // ts if ln > 0 else 0
        a = int(off[sg] - off[0]) + c0 * tb
        b = a + ln + c0 * ntl
        w0 = (a * nw + C - 1) // C
        we = min((b * nw + C - 1) // C, nw)
        for w in range(w0, we):
            lo = (w * C) // nw
            i = ((lo - a) + ts + c0 - 1) // (ts + c0)
            wt[2 * w] = tb + i if i < ntl else tb + ntl
            wt[2 * w + 1] = sg
    tbase[nseg] = NT
    return tbase, wt


def host_first_tiles(off, tb, ts, c0, nw):
    """The plans' host table (build_wave_table): first tile whose start cost
    is at least floor(w*C/nw), for w = 0..nw."""
    nseg = len(off) - 1
    C = int(off[nseg] - off[0]) + c0 * int(tb[nseg])
    cbase = lambda s: int(off[s] - off[0]) + c0 * int(tb[s])  # noqa: E731
    out = []
    a = 0
    for w in range(nw + 1):
        lo = (w * C) // nw
        while a + 1 < nseg and cbase(a + 1) <= lo:
            a += 1
        i = ((lo - cbase(a)) + ts + c0 - 1) // (ts + c0)
        out.append(int(tb[a]) + i if i < tb[a + 1] - tb[a] else int(tb[a + 1]))
    return out


def random_offsets(rng, nseg):
    kind = rng.integers(0, 3)
    if kind == 0:
        lens = rng.integers(0, 50, nseg)
    elif kind == 1:
        lens = np.floor(np.exp(rng.uniform(0, np.log(200000), nseg))).astype(np.int64)
    else:
        lens = rng.integers(0, 3, nseg) * rng.integers(0, 100000, nseg)  # many empty
    off = np.zeros(nseg + 1, dtype=np.int64)
    np.cumsum(lens, out=off[1:])
    return off


@pytest.mark.parametrize("seed", range(12))
def test_device_tables_cover_every_tile_once(seed):
    rng = np.random.default_rng(seed)
    nseg = int(rng.choice([1, 3, 1023, 1024, 1025, 2500, 5000]))
    off = random_offsets(rng, nseg)
    ts = int(rng.choice([256, 4096, 16384]))
    elem_bytes, dot = int(rng.choice([4, 8])), bool(rng.integers(0, 2))
    c0 = 16384 // (elem_bytes * (2 if dot else 1))
    nw = int(rng.choice([1, 4, 64, 1024]))
    tbase, wt = device_tables(off, ts, c0, nw)
    tiles = tiles_of(off, ts)
    assert np.array_equal(tbase[:-1], np.concatenate([[0], np.cumsum(tiles)[:-1]]))
    NT = int(tiles.sum())
    assert tbase[-1] == NT
    first = wt[0::2]
    assert np.all(first >= 0) and first[0] == 0 and first[-1] == NT
    assert np.all(np.diff(first) >= 0)  # the ranges tile [0, NT) in order
    for w in range(nw):
        t, sg = int(wt[2 * w]), int(wt[2 * w + 1])
        assert 0 <= sg < nseg
        if t < NT:
            seg_of_t = int(np.searchsorted(tbase, t, side="right") - 1)
            assert sg <= seg_of_t
    if NT > 0:
        assert list(first) == host_first_tiles(off, tbase, ts, c0, nw)


def test_no_tiles_gives_empty_ranges():
    off = np.zeros(5, dtype=np.int64)
    tbase, wt = device_tables(off, 4096, 1024, 8)
    assert tbase[-1] == 0 and np.all(wt[0::2] == 0)
