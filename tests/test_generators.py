"""The seeded input recipes: reproducible bits, values on their grids, the
sizes the workloads need."""
import hashlib

import numpy as np
import pytest

import oracle
import synth

DECADES = (6, 8, 10, 12, 14, 16)


def _h(*arrs):
    m = hashlib.sha256()
    for a in arrs:
        m.update(np.ascontiguousarray(a).tobytes())
    return m.hexdigest()[:16]


def test_uniform_reproducible_and_on_grid():
    for dtype, grid in ((np.float64, 2.0 ** 52), (np.float32, 2.0 ** 23)):
        a = synth.uniform(0, 1 << 16, dtype)
        b = synth.uniform(0, 1 << 16, dtype)
        assert _h(a) == _h(b)
        assert a.dtype == dtype and a.min() >= -1 and a.max() < 1
        k = (a.astype(np.float64) + 1.0) * grid
        assert np.all(k == np.floor(k))
        assert abs(float(a.mean())) < 0.02
    c = np.concatenate(list(synth.uniform_chunks(0, 1 << 16, np.float64, chunk=1000)))
    assert _h(c) == _h(synth.uniform(0, 1 << 16, np.float64))
    x, y = synth.uniform(5, 1000, np.float32, count=2)
    assert _h(x) == _h(synth.uniform(5, 1000, np.float32)) and _h(x) != _h(y)


def test_scaled_inputs():
    x, y = synth.scaled(2, 1 << 14)
    assert x.dtype == np.float32
    m, e = np.frexp(np.abs(x[x != 0]).astype(np.float64))
    assert e.min() >= -20 - 23 and e.max() <= 21
    # multiples of 2^-43: products and their remainders stay normal
    assert np.all(np.ldexp(x.astype(np.float64), 43) == np.floor(np.ldexp(x.astype(np.float64), 43)))


def test_segment_lengths_cfg():
    L = synth.segment_lengths(3, 20000)
    assert L.min() >= 1 and L.max() <= 1 << 20
    assert int(L.sum()) == 1504333896  # 20,000 log-uniform lengths, seed 3
    off = synth.offsets_from_lengths(L)
    assert off[0] == 0 and off[-1] == L.sum() and np.all(np.diff(off) == L)
    L2 = synth.segment_lengths(3, 20000, max_len=1 << 17)
    assert int(L2.sum()) == 221217512


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_illcond_reaches_its_decade(dtype):
    """At the configuration's N = 2^24, every target decade 1e6 .. 1e16 is
    reached within a factor of 10 (exact condition 2 sum|x y| / |sum x y|
    from the exact accumulator); the draws are reproducible."""
    for d in DECADES:
        x, y = synth.illcond_dot(synth.illcond_seed(d), 1 << 24, 10.0 ** d, dtype)
        ex = oracle.Exact(x, y)
        cond = 2 * ex.A / abs(ex.S)
        assert 10.0 ** (d - 1) < cond < 10.0 ** (d + 1), (d, cond)
        assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))
    x, y = synth.illcond_dot(synth.illcond_seed(8), 1 << 16, 1e8, dtype)
    x2, y2 = synth.illcond_dot(synth.illcond_seed(8), 1 << 16, 1e8, dtype)
    assert _h(x, y) == _h(x2, y2)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_illcond_low_block(dtype):
    """Below what the cancelling recipe reaches, the last n/16 elements are
    the non-cancelling block: every product there has the sign of the dot of
    the elements before it, and the earlier elements are the recipe's own
    (the block changes nothing before it)."""
    n = 1 << 16
    x, y = synth.illcond_dot(synth.illcond_seed(6), n, 1e6 / 64, dtype)
    x0, y0 = synth.illcond_dot(synth.illcond_seed(6), n, 1e6 / 64, dtype, low_block=False)
    m = n // 16
    head = oracle.Exact(x[:n - m], y[:n - m])
    p = x[n - m:].astype(np.float64) * y[n - m:].astype(np.float64)
    assert np.all(p * head.sign >= 0) and np.count_nonzero(p) > m // 2
    assert _h(x[:n // 2], y[:n // 2]) == _h(x0[:n // 2], y0[:n // 2])
    ex = oracle.Exact(x, y)
    cond = 2 * ex.A / abs(ex.S)
    assert 1e6 / 64 / 10 < cond < 1e6 / 64 * 10, cond


def test_hundred_hours_input():
    x = synth.hundred_hours()
    assert x.size == 3_600_000 and x.dtype == np.float32 and np.all(x == np.float32(0.1))


def test_permuted_illcond_keeps_the_exact_dot():
    import oracle
    for dtype in (np.float32, np.float64):
        x, y = synth.illcond_dot(synth.illcond_seed(12), 1 << 12, 1e12, dtype)
        px, py = synth.permute_pairs(synth.illcond_perm_seed(12), x, y)
        qx, qy = synth.permute_pairs(synth.illcond_perm_seed(12), x, y)
        assert np.array_equal(px, qx) and np.array_equal(py, qy)  # reproducible
        assert not np.array_equal(px, x)
        assert sorted((x.astype(np.float64) * y).tolist()) == sorted((px.astype(np.float64) * py).tolist())
        a, b = oracle.Exact(x, y), oracle.Exact(px, py)
        assert a.S == b.S and a.diff(a.S) == b.diff(a.S) and a.A == b.A


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_uniform_fill_is_the_serial_stream(dtype):
    """The threaded generator (jump-ahead per chunk) draws exactly the serial
    stream, for any thread count, across chunk boundaries and a ragged end."""
    n = (1 << 23) + 12345
    want = synth.uniform(3, n, dtype)
    for nt in (1, 3, 8):
        got = synth.uniform_fill(3, n, dtype, nthreads=nt)
        assert got.dtype == dtype and _h(got) == _h(want), nt
