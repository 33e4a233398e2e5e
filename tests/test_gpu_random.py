"""Seeded random sweep of GPU parity: every public mode and data type, sums
and dots, sizes from 0 to about 2^18, x and y at every position inside a
16-byte line, random launch shapes (single vector), random batches with
empty and tiny segments, random tiles and both the device-offset and plan
paths (segmented, every mode on both), and random multi-vector calls (1 to 64 vectors of mixed
lengths and alignments, explicit or default launch). Every pair must equal
the order model's bit for bit. Also data made of signed zeros, where only
the documented starting point (+0, +0) fixes the sign of the result."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1401_0248_amd as tf
import synth
from gpu_helpers import DEV, same_bits, to_dev

pytestmark = pytest.mark.gpu

FORMS = [(m, dot) for m in ("plain", "fast", "rigorous", "kahan") for dot in (False, True)] + \
        [("fast_rounded", True), ("rigorous_rounded", True), ("wide", False), ("wide", True),
         ("mixed", False), ("mixed", True)]
MULTI_MODES = ("plain", "fast", "rigorous", "kahan")  # plus the rounded dots


def _dtype_for(rng, mode):
    """The mixed form takes binary32 data only."""
    if mode == "mixed":
        return np.float32
    return (np.float32, np.float64)[rng.integers(0, 2)]


def _note(msg):
    print("[random] " + msg, file=sys.stderr, flush=True)


def _values(rng, n, dtype):
    kind = rng.integers(0, 3)
    if kind == 0:
        v = rng.standard_normal(n)
    elif kind == 1:
        v = rng.standard_normal(n) * np.exp2(rng.integers(-30, 30, n))
    else:
        v = np.round(rng.standard_normal(n) * 64) / 64  # many ties and exact sums
    return v.astype(dtype)


def _call(mode, dot, xd, yd, lc):
    if mode == "wide":
        return tf.dotd(xd, yd, lc) if dot else tf.sumd(xd, lc)
    if mode == "mixed":
        return tf.dot_mixed(xd, yd, lc) if dot else tf.sum_mixed(xd, lc)
    return tf.dot(xd, yd, mode, lc) if dot else tf.sum(xd, mode, lc)


@pytest.mark.parametrize("seed", range(16))
def test_random_single_vector(seed):
    rng = np.random.default_rng(1000 + seed)
    for case in range(40):
        mode, dot = FORMS[rng.integers(0, len(FORMS))]
        dtype = _dtype_for(rng, mode)
        W = 16 // np.dtype(dtype).itemsize
        n = int(np.floor(np.exp(rng.random() * np.log(1 << 18)))) if rng.random() < 0.9 else \
            int(rng.integers(0, 3))
        bt = int(rng.integers(1, 17)) * 64
        u = int(rng.choice([1, 2, 4, 8]))
        gb = int(rng.integers(1, 300))
        xs, ys = int(rng.integers(0, W)), int(rng.integers(0, W))
        x = _values(rng, n, dtype)
        y = _values(rng, n, dtype)
        xd, mis = to_dev(x, xs)
        yd, _ = to_dev(y, ys)
        got = _call(mode, dot, xd, yd, tf.Launch(bt, u, gb, 0, 0)).double().cpu().numpy()
        want = oracle.model_single(mode, x, y if dot else None, mis, bt, u, gb)
        assert same_bits(got, want), (seed, case, np.dtype(dtype).name, mode, dot, n, bt, u, gb,
                                      xs, ys)


@pytest.mark.parametrize("seed", range(12))
def test_random_segmented(seed):
    rng = np.random.default_rng(2000 + seed)
    for case in range(12):
        mode, dot = FORMS[rng.integers(0, len(FORMS))]
        dtype = _dtype_for(rng, mode)
        W = 16 // np.dtype(dtype).itemsize
        nseg = int(rng.integers(1, 400))
        lengths = np.floor(np.exp(rng.random(nseg) * np.log(1 << 14))).astype(np.int64)
        lengths[rng.random(nseg) < 0.15] = 0
        lengths[rng.random(nseg) < 0.15] = 1
        off = synth.offsets_from_lengths(lengths)
        n = int(off[-1])
        ts = 64 * W * int(rng.choice([1, 2, 4, 16, 64]))
        bt = int(rng.integers(1, 9)) * 64
        u = int(rng.choice([1, 2, 4, 8]))
        gb = int(rng.integers(1, 200))
        lc = tf.Launch(bt, u, gb, 0, ts)
        xs, ys = int(rng.integers(0, W)), int(rng.integers(0, W))
        x = _values(rng, n, dtype)
        y = _values(rng, n, dtype)
        xd, mis = to_dev(x, xs)
        yd, _ = to_dev(y, ys)
        want = oracle.model_seg(mode, x, off, y if dot else None, mis, u, ts)
        tdt = torch.float32 if dtype == np.float32 else torch.float64
        plan = tf.SegPlan(off, tdt, dot, mode, lc)
        got = plan.execute(xd, yd if dot else None).double().cpu().numpy()
        plan.close()
        tag = (seed, case, np.dtype(dtype).name, mode, dot, nseg, ts, bt, u, gb)
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), tag
        od = torch.from_numpy(np.asarray(off, dtype=np.int64)).to(DEV)
        if mode == "mixed":
            dev = tf.segdot_mixed(xd, yd, od, lc) if dot else tf.segsum_mixed(xd, od, lc)
        elif mode == "wide" and dtype == np.float32:
            dev = tf.segdotd(xd, yd, od, lc) if dot else tf.segsumd(xd, od, lc)
        else:
            dev = tf.segdot(xd, yd, od, mode, lc) if dot else tf.segsum(xd, od, mode, lc)
        got = dev.double().cpu().numpy()
        assert np.array_equal(got.view(np.uint64), want.view(np.uint64)), tag + ("device",)


@pytest.mark.parametrize("seed", range(8))
def test_random_multi(seed):
    rng = np.random.default_rng(3000 + seed)
    for case in range(6):
        dtype = (np.float32, np.float64)[rng.integers(0, 2)]
        dot = bool(rng.integers(0, 2))
        modes = MULTI_MODES + (("fast_rounded", "rigorous_rounded") if dot else ()) + ("wide",) + \
            (("mixed",) if dtype == np.float32 else ())
        mode = modes[rng.integers(0, len(modes))]
        W = 16 // np.dtype(dtype).itemsize
        count = int(rng.integers(1, tf.MAX_MULTI + 1))
        lengths = np.floor(np.exp(rng.random(count) * np.log(1 << 17))).astype(np.int64)
        lengths[rng.random(count) < 0.1] = 0
        lengths[rng.random(count) < 0.1] = 1
        if rng.random() < 0.7:
            bt, u, gb = int(rng.integers(1, 17)) * 64, int(rng.choice([1, 2, 4, 8])), \
                int(rng.integers(1, 300))
            lc = tf.Launch(bt, u, gb, 0, 0)
        else:
            lc = None
            d = tf.default_launch(0, np.dtype(dtype).itemsize, dot, mode, int(lengths.max()))
            bt, u, gb = d.block_threads, d.unroll, d.grid_blocks
        hx, hy, dx, dy, mis = [], [], [], [], []
        for v in range(count):
            n = int(lengths[v])
            x, y = _values(rng, n, dtype), _values(rng, n, dtype)
            xd, m = to_dev(x, int(rng.integers(0, W)))
            yd, _ = to_dev(y, int(rng.integers(0, W)))
            hx.append(x)
            hy.append(y)
            dx.append(xd)
            dy.append(yd)
            mis.append(m)
        if mode == "wide":
            out = tf.multidotd(dx, dy, lc) if dot else tf.multisumd(dx, lc)
        elif mode == "mixed":
            out = tf.multidot_mixed(dx, dy, lc) if dot else tf.multisum_mixed(dx, lc)
        else:
            out = tf.multidot(dx, dy, mode, lc) if dot else tf.multisum(dx, mode, lc)
        out = out.double().cpu().numpy()
        for v in range(count):
            want = oracle.model_single(mode, hx[v], hy[v] if dot else None, mis[v], bt, u, gb)
            assert same_bits(tuple(out[v]), want), (seed, case, np.dtype(dtype).name, mode, dot,
                                                    count, v, int(lengths[v]), bt, u, gb)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_signed_zeros(dtype):
    """All -0: every chain starts at +0 and +0 + (-0) = +0, so the value is
    +0, not the -0 a sequence of -0 additions alone would give. Mixed zeros
    and products of zeros with negative numbers give the model's signs."""
    rng = np.random.default_rng(5)
    for n in (1, 7, 1000, 70000):
        x = np.full(n, -0.0, dtype=dtype)
        y = np.where(rng.random(n) < 0.5, -1.0, 1.0).astype(dtype)
        y[rng.random(n) < 0.3] = -0.0
        xd, mis = to_dev(x, 1)
        yd, _ = to_dev(y, 0)
        for mode, dot in FORMS:
            if mode == "mixed" and dtype == np.float64:
                continue
            lc = tf.Launch(128, 2, 3, 0, 0)
            got = _call(mode, dot, xd, yd, lc).double().cpu().numpy()
            want = oracle.model_single(mode, x, y if dot else None, mis, 128, 2, 3)
            assert same_bits(got, want), (n, mode, dot)
            if not dot:
                assert got[0] == 0.0 and not np.signbit(got[0]), (n, mode)
