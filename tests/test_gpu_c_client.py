"""A native client of the C ABI (tests/c_client/client.cpp, built by
__graft_entry__.build()): no Python or torch between it and the library.
Its printed results must equal the oracle's, bit for bit: the order model
in the default launches the library reports, and the monitor's flag rule.
The inputs are the client's closed-form arrays, rebuilt here."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
from oracle import monitor
from paper_1401_0248_amd import _lib
from paper_1401_0248_amd._lib import Launch

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "client")
N = 1000003
OFF = np.array([0, 10, 10, 1000, N], dtype=np.int64)


def _inputs():
    i = np.arange(N, dtype=np.int64)
    x = 1.0 + (i % 1000).astype(np.float64) * 2.0 ** -40
    y = ((7 * i) % 201 - 100).astype(np.float64) / 32.0
    xf = (1.0 + (i % 1000).astype(np.float64) * 2.0 ** -20).astype(np.float32)
    return x, y, xf


def _launch(kind, dtype, is_dot, mode, n, nseg=0):
    lc = Launch()
    assert _lib.load().twofold_default_launch(kind, dtype, is_dot, mode, n, nseg,
                                              ctypes.byref(lc)) == 0
    return lc


def _run():
    assert os.path.exists(BIN), "native client not built: run __graft_entry__.build()"
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    rows = {}
    for line in r.stdout.splitlines():
        f = line.split()
        rows[f[0]] = f[1:]
    return rows


def _pair(row):
    assert int(row[0]) == 0, row
    return float.fromhex(row[1]), float.fromhex(row[2])


def test_native_client_matches_the_oracle():
    rows = _run()
    x, y, xf = _inputs()
    mis = 0  # hipMalloc returns 256-byte aligned memory
    lc = _launch(0, 8, 0, 2, N)
    want = oracle.model_single("rigorous", x, None, mis, lc.block_threads, lc.unroll, lc.grid_blocks)
    got = _pair(rows["sum_f64_rigorous"])
    assert got == (want[0], want[1])
    assert oracle.Exact(x).diff(*got) == 0.0  # grid data: value + error is the exact sum
    lc = _launch(0, 8, 0, 0, N)
    want = oracle.model_single("plain", x, None, mis, lc.block_threads, lc.unroll, lc.grid_blocks)
    assert _pair(rows["sum_f64_plain"]) == (want[0], want[1])
    lc = _launch(0, 8, 1, 2, N)
    want = oracle.model_single("rigorous", x, y, mis, lc.block_threads, lc.unroll, lc.grid_blocks)
    assert _pair(rows["dot_f64_rigorous"]) == (want[0], want[1])
    lc = _launch(0, 4, 0, 1, N)
    want = oracle.model_single("fast", xf, None, mis, lc.block_threads, lc.unroll, lc.grid_blocks)
    assert _pair(rows["sum_f32_fast"]) == (want[0], want[1])
    lc = _launch(1, 8, 1, 2, N, 4)
    seg = oracle.model_seg("rigorous", x, OFF, y, mis, lc.unroll, lc.tile_elems)
    for s in range(4):
        assert _pair(rows["segdot_f64_rigorous_%d" % s]) == (seg[s][0], seg[s][1]), s
    assert tuple(seg[1]) == (0.0, 0.0)
    # the multi-vector call: each row is the order model's single-vector
    # result under the default launch of the longest vector
    lc = _launch(0, 8, 1, 2, N)
    for v, (a, n) in enumerate(((0, N), (1, N - 1), (0, 1000))):
        want = oracle.model_single("rigorous", x[a:a + n], y[a:a + n], a % 2, lc.block_threads,
                                   lc.unroll, lc.grid_blocks)
        assert _pair(rows["multidot_f64_rigorous_%d" % v]) == (want[0], want[1]), v
    # binary64 results: the mixed-form dot, double-word sums in one call
    lc = _launch(0, 4, 1, 7, N)
    want = oracle.model_single("mixed", xf, xf, mis, lc.block_threads, lc.unroll, lc.grid_blocks)
    assert _pair(rows["dot_mixed_f32"]) == (want[0], want[1])
    lc = _launch(0, 8, 0, 3, N)
    for v, a in enumerate((0, 1)):
        want = oracle.model_single("wide", x[a:], None, a % 2, lc.block_threads, lc.unroll,
                                   lc.grid_blocks)
        assert _pair(rows["multisumd_f64_%d" % v]) == (want[0], want[1]), v
    # the mixed batch: its launch is the default of its largest item (the
    # binary64 dot); each pair is the single call's with that launch
    lc = _launch(0, 8, 1, 2, N)
    for row, mode, a, b in (("batch_dot_f64_rigorous", "rigorous", x, y),
                            ("batch_sum_f32_fast", "fast", xf, None)):
        want = oracle.model_single(mode, a, b, mis, lc.block_threads, lc.unroll, lc.grid_blocks)
        assert _pair(rows[row]) == (want[0], want[1]), row
    m = rows["monitor"]
    assert int(m[0]) == 0
    flags = monitor.flags(seg, np.diff(OFF), 0.0, np.float64)
    assert [int(v) for v in m[1:5]] == flags
    assert int(m[5]) == sum(1 for f in flags if f)
