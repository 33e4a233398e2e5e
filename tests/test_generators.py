"""The seeded input recipes: reproducible bits, values on their grids, the
sizes the workloads need."""
import hashlib

import numpy as np
import pytest

import oracle
import synth


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
    for d in (6, 10, 16):
        x, y = synth.illcond_dot(synth.illcond_seed(d), 1 << 16, 10.0 ** d, dtype)
        ex = oracle.Exact(x, y)
        cond = 2 * ex.A / abs(ex.S)
        assert 10.0 ** (d - 1.5) < cond < 10.0 ** (d + 1.5), (d, cond)
        x2, y2 = synth.illcond_dot(synth.illcond_seed(d), 1 << 16, 10.0 ** d, dtype)
        assert _h(x, y) == _h(x2, y2)
        assert np.all(np.isfinite(x)) and np.all(np.isfinite(y))


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
