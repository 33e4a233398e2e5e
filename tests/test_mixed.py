"""Pins of the oracle's mixed mode (binary32 data, the rigorous form with a
binary64 error term), independent of the GPU library:

* the value is the binary32 rigorous value of the same order, bit for bit
  (the value path is the same arithmetic);
* on exact-grid data value + error is the exact sum;
* every result lies within the bound of its own tree (oracle.bounds.
  mixed_bound), which is far below what the binary32 error term allows, so
  an error term summed in binary32, a dropped product remainder or a wrong
  sign fails it;
* the paper's "100 hours" ticks (section "Examples"): the binary32 twofold
  result is off by about 0.06 hours sequentially; the mixed result is
  within the bound of the exact sum.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import bounds

LAUNCHES = [(256, 1, 1), (256, 4, 3), (512, 2, 2), (1024, 8, 5), (64, 1, 1), (128, 2, 7)]

_DATA = {}


def _datasets(n, seed):
    key = (n, seed)
    if key not in _DATA:
        _DATA[key] = [("uniform",) + tuple(synth.uniform(seed, n, np.float32, count=2)),
                      ("illcond",) + tuple(synth.illcond_dot(synth.illcond_seed(16), n, 1e16,
                                                             np.float32)),
                      ("scaled",) + tuple(synth.scaled(seed, n))]
    return _DATA[key]


@pytest.mark.parametrize("launch", LAUNCHES)
def test_mixed_value_is_the_rigorous_value(launch):
    bt, U, gb = launch
    for name, x, y in _datasets(1 << 13, 3):
        for yy in (None, y):
            for mis in (0, 3):
                m = oracle.model_single("mixed", x, yy, mis, bt, U, gb)
                r = oracle.model_single("rigorous", x, yy, mis, bt, U, gb)
                assert np.float64(m[0]).tobytes() == np.float64(r[0]).tobytes(), name
                assert float(np.float32(m[0])) == m[0]  # a binary32 number


@pytest.mark.parametrize("launch", LAUNCHES)
def test_mixed_within_its_tree_bound(launch):
    bt, U, gb = launch
    n = 1 << 14
    for name, x, y in _datasets(n, 7):
        for yy in (None, y):
            ex = oracle.Exact(x, yy)
            got = oracle.model_single("mixed", x, yy, 1, bt, U, gb)
            Lc, D = bounds.single_depths(np.float32, n, bt, U, gb)
            b = bounds.mixed_bound(Lc, D, ex.A)
            assert abs(ex.diff(got[0], got[1])) <= b, (name, yy is None)
            # the bound is far tighter than the binary32 rigorous one
            assert b < 1e-6 * bounds.single_bound(np.float32, n, bt, U, gb, ex.A)


def test_mixed_exact_grid():
    for n in (0, 1, 7, 1000, 65536 + 3):
        x = synth.uniform(n + 31, n, np.float32)
        ex = oracle.Exact(x)
        for bt, U, gb in LAUNCHES[:3]:
            got = oracle.model_single("mixed", x, None, 2, bt, U, gb)
            assert ex.diff(got[0], got[1]) == 0.0, (n, got)


def test_mixed_beats_the_binary32_error_term():
    """On ill-conditioned binary32 dots the binary32 rigorous result errs by
    about u^2 sum|x y|; the mixed one, at least a thousand times less."""
    x, y = synth.illcond_dot(synth.illcond_seed(16), 1 << 16, 1e16, np.float32)
    ex = oracle.Exact(x, y)
    r = oracle.model_single("rigorous", x, y, 0, 256, 4, 16)
    m = oracle.model_single("mixed", x, y, 0, 256, 4, 16)
    wide = oracle.model_single("wide", x, y, 0, 256, 4, 16)  # binary64 plain on the same data
    assert abs(ex.diff(*m)) * 1e3 <= abs(ex.diff(*r))
    assert abs(ex.diff(*m)) <= abs(ex.diff(*wide))


def test_hundred_hours_ticks():
    """3,600,000 ticks of 0.1f seconds (the paper's example): the sequential
    binary32 twofold sum misses the exact total by about 0.064 hours; the
    mixed result of a GPU-order launch is within its bound of it."""
    n = 3600000
    x = np.full(n, np.float32(0.1), dtype=np.float32)
    ex = oracle.Exact(x)
    v, e = oracle.seq("sumt", x)
    assert abs(ex.diff(float(v), float(e))) / 3600 > 0.06
    for bt, U, gb in ((64, 1, 1), (256, 4, 64)):
        got = oracle.model_single("mixed", x, None, 0, bt, U, gb)
        Lc, D = bounds.single_depths(np.float32, n, bt, U, gb)
        assert abs(ex.diff(*got)) <= bounds.mixed_bound(Lc, D, ex.A)
        assert abs(ex.diff(*got)) / 3600 < 1e-12


def test_mixed_segments():
    ts = 64 * 4 * 2
    lengths = synth.segment_lengths(6, 60, max_len=1 << 13)
    off = synth.offsets_from_lengths(lengths)
    n = int(off[-1])
    x, y = synth.illcond_dot(synth.illcond_seed(12), max(4, n + n % 2), 1e12, np.float32)
    x, y = x[:n], y[:n]
    got = oracle.model_seg("mixed", x, off, y, 1, 2, ts)
    rig = oracle.model_seg("rigorous", x, off, y, 1, 2, ts)
    for s in range(len(lengths)):
        a, b = off[s], off[s + 1]
        assert got[s][0] == rig[s][0], s
        ex = oracle.Exact(x[a:b], y[a:b])
        Lc, D = bounds.segment_depths(np.float32, b - a, ts)
        assert abs(ex.diff(*got[s])) <= bounds.mixed_bound(Lc, D, ex.A), s


def test_mixed_only_for_binary32():
    x = np.ones(10)
    with pytest.raises(Exception):
        oracle.model_single("mixed", x, None, 0, 64, 1, 1)
