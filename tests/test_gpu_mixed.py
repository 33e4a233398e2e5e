"""GPU parity of the mixed form (binary32 data, rigorous twofold with a
binary64 error term): bitwise against the order model for explicit launch
shapes, single-vector and plans; the value bitwise the binary32 rigorous
value; results within the mixed tree bound of the exact sum."""
import numpy as np
import pytest
import torch

import oracle
import paper_1401_0248_amd as tf
import synth
from gpu_helpers import DEV, launch, pair, same_bits, to_dev
from oracle import bounds

pytestmark = pytest.mark.gpu

SIZES = [0, 1, 3, 17, 1000, 4097, 65536 + 5, (1 << 20) + 3]
LAUNCHES = [(256, 1, 1), (256, 4, 7), (512, 2, 3), (1024, 8, 5), (256, 4, 300), (64, 2, 2),
            (128, 8, 33)]


def _data(seed, n):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(n) * np.exp2(rng.integers(-10, 10, n))).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    return x, y


@pytest.mark.parametrize("is_dot", [False, True])
def test_mixed_bitwise_vs_model(is_dot):
    for n in SIZES:
        x, y = _data(n + 5, n)
        for li, (bt, u, gb) in enumerate(LAUNCHES):
            xd, mis = to_dev(x, li % 4)
            yd, _ = to_dev(y, (li + li % 2) % 4) if is_dot else (None, 0)
            lc = launch(bt, u, gb)
            got = tf.dot_mixed(xd, yd, lc) if is_dot else tf.sum_mixed(xd, lc)
            assert got.dtype == torch.float64
            want = oracle.model_single("mixed", x, y if is_dot else None, mis, bt, u, gb)
            assert same_bits(pair(got), want), (n, bt, u, gb, pair(got), list(want))
            rig = tf.dot(xd, yd, "rigorous", lc) if is_dot else tf.sum(xd, "rigorous", lc)
            assert pair(got)[0] == pair(rig)[0]  # the binary32 rigorous value


def test_mixed_plans_vs_model():
    lengths = synth.segment_lengths(8, 300, max_len=1 << 15)
    off = synth.offsets_from_lengths(lengths)
    n = int(off[-1])
    x, y = _data(9, n)
    xd, mis = to_dev(x, 1)
    yd, _ = to_dev(y, 1)
    for u, ts in ((2, 2048), (4, 8192), (8, 4096)):
        lc = launch(256, u, 16, ts)
        for is_dot in (False, True):
            plan = tf.SegPlan(off, torch.float32, is_dot, "mixed", lc)
            got = plan.execute(xd, yd if is_dot else None)
            assert got.dtype == torch.float64
            want = oracle.model_seg("mixed", x, off, y if is_dot else None, mis, u, ts)
            g = got.cpu().numpy()
            assert np.array_equal(g.view(np.uint64), np.asarray(want).view(np.uint64)), (u, ts)


def test_mixed_default_launch_accuracy():
    """Ill-conditioned binary32 dot (N = 2^20, target condition 1e16), the
    tuned default launch: within the mixed bound of its tree, and more
    accurate than binary64 plain summation of the same binary32 data."""
    n = 1 << 20
    x, y = synth.illcond_dot(synth.illcond_seed(16), n, 1e16, np.float32)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.from_numpy(y).to(DEV)
    got = pair(tf.dot_mixed(xd, yd))
    ex = oracle.Exact(x, y)
    lc = tf.default_launch(0, 4, True, "mixed", n)
    Lc, D = bounds.single_depths(np.float32, n, lc.block_threads, lc.unroll, lc.grid_blocks)
    assert abs(ex.diff(*got)) <= bounds.mixed_bound(Lc, D, ex.A)
    d = pair(tf.dotd(xd, yd))
    assert abs(ex.diff(*got)) <= abs(ex.diff(*d))


def test_mixed_rejects_binary64_data():
    x = torch.ones(16, dtype=torch.float64, device=DEV)
    with pytest.raises(TypeError):
        tf.sum_mixed(x)
    with pytest.raises(tf.TwofoldError):
        tf.sum(x.float(), "mixed")


def test_mixed_tiny_sizes():
    e = torch.empty(0, dtype=torch.float32, device=DEV)
    got = tf.sum_mixed(e).cpu().numpy()
    assert got.dtype == np.float64 and np.array_equal(got.view(np.uint64), np.zeros(2, np.uint64))
    x = torch.tensor([0.1], dtype=torch.float32, device=DEV)
    y = torch.tensor([3.0], dtype=torch.float32, device=DEV)
    assert pair(tf.sum_mixed(x)) == (float(np.float32(0.1)), 0.0)
    # one product: value fl32(x*y), error its exact remainder
    p = np.float32(0.1) * np.float32(3.0)
    rem = float(np.float64(np.float32(0.1)) * 3.0 - np.float64(p))
    assert pair(tf.dot_mixed(x, y)) == (float(p), rem)
