"""GPU parity of the multi-vector calls (twofold_multisum_* /
twofold_multidot_*, and the binary64-result forms twofold_multisumd_*,
twofold_multidotd_*, twofold_multi{sum,dot}_mixed_f32): every row is bitwise the order model's single-vector
result for that vector under the call's launch, and bitwise the
single-vector call with the same launch, whatever the other vectors' lengths
and alignments, and whether the vectors run side by side (short ones) or
one after another (long ones)."""
import numpy as np
import pytest
import torch

import oracle
import paper_1401_0248_amd as tf
from gpu_helpers import launch, pair, same_bits, to_dev

pytestmark = pytest.mark.gpu

LAUNCHES = [(256, 1, 1), (256, 4, 7), (512, 2, 3), (64, 2, 2), (128, 8, 33), (256, 4, 300)]
LENGTHS = [0, 1, 3, 17, 1000, 4097, 65536 + 5, 100003]
SHIFTS = [0, 1, 3, 2]


def _data(seed, n, dtype):
    rng = np.random.default_rng(seed)
    x = (rng.standard_normal(n) * np.exp2(rng.integers(-10, 10, n))).astype(dtype)
    y = rng.standard_normal(n).astype(dtype)
    return x, y


def _vectors(dtype, is_dot, lengths, seed):
    """Host arrays and device views; vector v starts `SHIFTS[v % 4]` elements
    past a 256-byte boundary, y one further for odd v (x and y then sit at
    different positions in their 16-byte lines)."""
    hx, hy, dx, dy, mis = [], [], [], [], []
    for v, n in enumerate(lengths):
        x, y = _data(seed + v, n, dtype)
        xd, m = to_dev(x, SHIFTS[v % 4])
        hx.append(x)
        dx.append(xd)
        mis.append(m)
        if is_dot:
            yd, _ = to_dev(y, SHIFTS[v % 4] + (v % 2))
            hy.append(y)
            dy.append(yd)
    return hx, (hy if is_dot else None), dx, (dy if is_dot else None), mis


def _call(dx, dy, mode, lc=None):
    return tf.multidot(dx, dy, mode, lc) if dy is not None else tf.multisum(dx, mode, lc)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("is_dot", [False, True])
@pytest.mark.parametrize("mode", ["plain", "fast", "rigorous", "kahan"])
def test_multi_bitwise_vs_model(dtype, is_dot, mode):
    hx, hy, dx, dy, mis = _vectors(dtype, is_dot, LENGTHS, 100)
    for bt, u, gb in LAUNCHES:
        out = _call(dx, dy, mode, launch(bt, u, gb)).cpu().numpy().astype(np.float64)
        for v in range(len(LENGTHS)):
            want = oracle.model_single(mode, hx[v], hy[v] if is_dot else None, mis[v], bt, u, gb)
            assert same_bits(tuple(out[v]), want), (v, LENGTHS[v], bt, u, gb, tuple(out[v]),
                                                    list(want))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("mode", ["fast_rounded", "rigorous_rounded"])
def test_multi_rounded_dots_vs_model(dtype, mode):
    hx, hy, dx, dy, mis = _vectors(dtype, True, LENGTHS, 200)
    for bt, u, gb in LAUNCHES[1::2]:
        out = tf.multidot(dx, dy, mode, launch(bt, u, gb)).cpu().numpy().astype(np.float64)
        for v in range(len(LENGTHS)):
            want = oracle.model_single(mode, hx[v], hy[v], mis[v], bt, u, gb)
            assert same_bits(tuple(out[v]), want), (v, bt, u, gb)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("is_dot", [False, True])
@pytest.mark.parametrize("longest", [(1 << 22) + 5, (1 << 24) + 9])
def test_multi_equals_single_calls_default_launch(dtype, is_dot, longest):
    # several ill-sized long vectors: the default launch is the longest one's,
    # and every row equals the single call made with that launch. Vectors
    # that read up to 64 MiB run side by side, longer ones one after another
    # (2^24 + 9 elements take the second way for every type and operation)
    lengths = [longest, (1 << 21) + 3, 0, 12345, 1 << 22]
    _, _, dx, dy, _ = _vectors(dtype, is_dot, lengths, 300)
    for mode in ("fast", "rigorous"):
        out = _call(dx, dy, mode)
        lc = tf.default_launch(0, np.dtype(dtype).itemsize, is_dot, mode, max(lengths))
        for v in range(len(lengths)):
            one = tf.dot(dx[v], dy[v], mode, lc) if is_dot else tf.sum(dx[v], mode, lc)
            assert torch.equal(out[v].view(torch.int8), one.view(torch.int8)), (mode, v)


def _wide_call(form, dx, dy, lc=None):
    if form == "wide":
        return tf.multidotd(dx, dy, lc) if dy is not None else tf.multisumd(dx, lc)
    return tf.multidot_mixed(dx, dy, lc) if dy is not None else tf.multisum_mixed(dx, lc)


def _wide_single(form, x, y, lc):
    if form == "wide":
        return tf.dotd(x, y, lc) if y is not None else tf.sumd(x, lc)
    return tf.dot_mixed(x, y, lc) if y is not None else tf.sum_mixed(x, lc)


@pytest.mark.parametrize("dtype,form", [(np.float32, "wide"), (np.float64, "wide"),
                                        (np.float32, "mixed")])
@pytest.mark.parametrize("is_dot", [False, True])
def test_multi_wide_and_mixed_vs_model(dtype, form, is_dot):
    """The binary64-result forms (binary64 accumulator for binary32 data,
    double-word for binary64 data, the mixed form): every row bitwise the
    order model's and the single-vector call's under the same launch."""
    hx, hy, dx, dy, mis = _vectors(dtype, is_dot, LENGTHS, 500)
    for bt, u, gb in LAUNCHES[::2] + [LAUNCHES[1]]:
        lc = launch(bt, u, gb)
        out = _wide_call(form, dx, dy, lc)
        assert out.dtype == torch.float64
        got = out.cpu().numpy()
        for v in range(len(LENGTHS)):
            want = oracle.model_single(form, hx[v], hy[v] if is_dot else None, mis[v], bt, u, gb)
            assert same_bits(tuple(got[v]), want), (v, LENGTHS[v], bt, u, gb)
            one = _wide_single(form, dx[v], dy[v] if is_dot else None, lc)
            assert torch.equal(out[v].view(torch.int8), one.view(torch.int8)), v


@pytest.mark.parametrize("dtype,form", [(np.float32, "wide"), (np.float64, "wide"),
                                        (np.float32, "mixed")])
def test_multi_wide_and_mixed_default_launch(dtype, form):
    # long vectors in turn (2^24 + 9 binary64 elements read more than 64 MiB)
    # and short ones side by side, each against its single call
    for lengths in ([(1 << 24) + 9, 12345, 0, 1 << 20], [(1 << 20) + 3, 1000, 1 << 19]):
        _, _, dx, dy, _ = _vectors(dtype, True, lengths, 600)
        out = _wide_call(form, dx, dy)
        lc = tf.default_launch(0, np.dtype(dtype).itemsize, True, form, max(lengths))
        for v in range(len(lengths)):
            one = _wide_single(form, dx[v], dy[v], lc)
            assert torch.equal(out[v].view(torch.int8), one.view(torch.int8)), (lengths, v)


def test_multi_64_vectors_and_graph_replay():
    lengths = [(v * 7919) % 5000 for v in range(64)]
    hx, hy, dx, dy, mis = _vectors(np.float64, True, lengths, 400)
    lc = launch(256, 2, 4)
    out = torch.empty((64, 2), dtype=torch.float64, device="cuda:0")
    tf.multidot(dx, dy, "rigorous", lc, out=out)
    eager = out.clone()
    for v in range(64):
        want = oracle.model_single("rigorous", hx[v], hy[v], mis[v], 256, 2, 4)
        assert same_bits(pair(out[v]), want), v
    s = torch.cuda.Stream()
    ws = tf.Workspace(1 << 16, "cuda:0")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        tf.multidot(dx, dy, "rigorous", lc, out=out, ws=ws)
    for _ in range(3):
        out.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out.view(torch.int8), eager.view(torch.int8))


def test_multi_rejects_bad_input():
    x = torch.zeros(100, dtype=torch.float32, device="cuda:0")
    with pytest.raises(ValueError):
        tf.multisum([x] * 65)
    with pytest.raises(ValueError):
        tf.multisum([x, x.double()])
    with pytest.raises(tf.TwofoldError):
        tf.multisum([x], "wide")  # binary64 rows: multisumd
    with pytest.raises(tf.TwofoldError):
        tf.multisum([x], "mixed")  # binary64 rows: multisum_mixed
    with pytest.raises(TypeError):
        tf.multisum_mixed([x.double()])
    with pytest.raises(ValueError):  # binary64 rows do not fit a binary32 out
        tf.multisumd([x, x], out=torch.empty((2, 2), dtype=torch.float32, device="cuda:0"))
    with pytest.raises(ValueError):
        tf.multisum([x, x], out=torch.empty((1, 2), dtype=torch.float32, device="cuda:0"))
    with pytest.raises(tf.TwofoldError):
        tf.multidot([x[1:]], [x[:-1]], "rigorous", launch(100, 4, 1))


def test_multi_empty_and_single_element_vectors():
    # every vector empty: (+0, +0) each, whatever the launch
    e = torch.empty(0, dtype=torch.float64, device="cuda:0")
    for lc in (None, launch(256, 4, 7)):
        out = tf.multidot([e, e, e], [e, e, e], "rigorous", lc).cpu().numpy()
        assert np.array_equal(out.view(np.uint64), np.zeros((3, 2), dtype=np.uint64))
    # one element each: a sum gives (x, +0), a rigorous dot (p, pi) exactly
    xs = [torch.tensor([v], dtype=torch.float64, device="cuda:0") for v in (1.5, -2.0 ** -40, 3.0)]
    ys = [torch.tensor([v], dtype=torch.float64, device="cuda:0") for v in (1.0 / 3, 7.0, -0.1)]
    s = tf.multisum(xs, "rigorous").cpu().numpy()
    assert [tuple(r) for r in s] == [(1.5, 0.0), (-2.0 ** -40, 0.0), (3.0, 0.0)]
    d = tf.multidot(xs, ys, "rigorous").cpu().numpy()
    for v in range(3):
        a, b = float(xs[v][0]), float(ys[v][0])
        p = a * b
        pi = float(np.float64(oracle.seq("dott", np.array([a]), np.array([b]))[1]))
        assert (d[v][0], d[v][1]) == (p, pi), v
