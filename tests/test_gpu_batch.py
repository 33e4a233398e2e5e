"""GPU parity of the mixed batch (twofold_batch): items of both data types,
sums and dots, every mode (the binary64-result ones too), ragged lengths
and alignments. Every item's pair is bitwise the order model's
single-vector result under the batch's launch and bitwise the single call
with that launch, whether the items run side by side or in turn."""
import numpy as np
import pytest
import torch

import oracle
import paper_1401_0248_amd as tf
from gpu_helpers import launch, same_bits, to_dev

pytestmark = pytest.mark.gpu

MODES_SUM = ("plain", "fast", "rigorous", "kahan")
MODES_DOT = MODES_SUM + ("fast_rounded", "rigorous_rounded")


def _items(seed, count, max_len, wide=False):
    rng = np.random.default_rng(seed)
    host, dev = [], []
    for v in range(count):
        dtype = (np.float32, np.float64)[rng.integers(0, 2)]
        dot = bool(rng.integers(0, 2))
        mode = (MODES_DOT if dot else MODES_SUM)[rng.integers(0, 6 if dot else 4)]
        if wide and rng.random() < 0.4:  # the binary64-result forms
            mode = "mixed" if (dtype == np.float32 and rng.random() < 0.5) else "wide"
        n = int(rng.choice([0, 1, 3, 17, 1000, 4097, int(rng.integers(1, max_len))]))
        x = (rng.standard_normal(n) * np.exp2(rng.integers(-12, 12, n))).astype(dtype)
        y = rng.standard_normal(n).astype(dtype)
        W = 16 // np.dtype(dtype).itemsize
        xd, mis = to_dev(x, int(rng.integers(0, W)))
        yd = to_dev(y, int(rng.integers(0, W)))[0] if dot else None
        host.append((x, y if dot else None, mode, mis))
        dev.append((xd, yd, mode))
    return host, dev


def _single(xd, yd, mode, lc):
    if mode == "wide":
        return tf.dotd(xd, yd, lc) if yd is not None else tf.sumd(xd, lc)
    if mode == "mixed":
        return tf.dot_mixed(xd, yd, lc) if yd is not None else tf.sum_mixed(xd, lc)
    return tf.dot(xd, yd, mode, lc) if yd is not None else tf.sum(xd, mode, lc)


@pytest.mark.parametrize("seed,wide", [(s, w) for s in range(4) for w in (False, True)])
def test_batch_bitwise_vs_model_and_single_calls(seed, wide):
    host, dev = _items(100 + seed, 40, 1 << 17, wide)
    for bt, u, gb in ((256, 1, 1), (256, 4, 7), (512, 2, 3), (128, 8, 33)):
        lc = launch(bt, u, gb)
        outs = tf.batch(dev, lc)
        for v, ((x, y, mode, mis), (xd, yd, _)) in enumerate(zip(host, dev)):
            want = oracle.model_single(mode, x, y, mis, bt, u, gb)
            got = outs[v].double().cpu().numpy()
            assert same_bits(tuple(got), want), (seed, v, mode, x.dtype, x.size, bt, u, gb)
            assert torch.equal(outs[v].view(torch.int8), _single(xd, yd, mode, lc).view(torch.int8)), \
                (seed, v)


def test_batch_default_launch_long_items_in_turn():
    # items above 64 MiB run in turn through one block set; the launch is the
    # default of the item that reads the most (the binary64 dot)
    N = 1 << 24
    x64 = torch.empty(N + 3, dtype=torch.float64, device="cuda:0").uniform_(-1, 1)
    y64 = torch.empty(N + 3, dtype=torch.float64, device="cuda:0").uniform_(-1, 1)
    x32 = x64.float()
    y32 = y64.float()
    items = [(x64[:N], y64[:N], "rigorous"), (x32, y32, "fast"), (x64[1:], None, "kahan"),
             (x32[:1000], None, "plain"), (x64[2:N + 2], y64[1:N + 1], "fast")]
    outs = tf.batch(items)
    lc = tf.default_launch(0, 8, True, "rigorous", N)
    for v, (x, y, mode) in enumerate(items):
        one = tf.dot(x, y, mode, lc) if y is not None else tf.sum(x, mode, lc)
        assert torch.equal(outs[v].view(torch.int8), one.view(torch.int8)), v


def test_batch_default_launch_caps_the_unroll():
    # the largest item, a binary32 sum of 2^26 elements, has a default launch
    # of eight vectors a round; the batch takes at most four
    n = 1 << 26
    x = torch.empty(n, dtype=torch.float32, device="cuda:0").uniform_(-1, 1)
    y = torch.empty(1000, dtype=torch.float64, device="cuda:0").uniform_(-1, 1)
    d = tf.default_launch(0, 4, False, "rigorous", n)
    lc = tf.Launch(d.block_threads, min(d.unroll, 4), d.grid_blocks, 0, 0)
    outs = tf.batch([(x, None, "rigorous"), (y, y, "fast")])
    assert torch.equal(outs[0].view(torch.int8), tf.sum(x, "rigorous", lc).view(torch.int8))
    assert torch.equal(outs[1].view(torch.int8), tf.dot(y, y, "fast", lc).view(torch.int8))


def test_batch_graph_replay():
    host, dev = _items(7, 24, 1 << 15)
    lc = launch(256, 2, 4)
    outs = [torch.empty(2, dtype=xd.dtype, device="cuda:0") for xd, _, _ in dev]
    tf.batch(dev, lc, outs=outs)
    eager = [o.clone() for o in outs]
    s = torch.cuda.Stream()
    ws = tf.Workspace(1 << 16, "cuda:0")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        tf.batch(dev, lc, outs=outs, ws=ws)
    for _ in range(3):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            assert torch.equal(o.view(torch.int8), e.view(torch.int8))


def test_batch_rejects_bad_items():
    x = torch.zeros(100, dtype=torch.float32, device="cuda:0")
    with pytest.raises(tf.TwofoldError):
        tf.batch([(x.double(), x.double(), "mixed")])  # the mixed form: binary32 data
    with pytest.raises(tf.TwofoldError):
        tf.batch([(x, None, "fast_rounded")])
    with pytest.raises(ValueError):
        tf.batch([(x, None, "fast")] * 65)
    with pytest.raises(ValueError):
        tf.batch([(x, None, "fast")], outs=[torch.empty(2, dtype=torch.float64, device="cuda:0")])
