"""GPU parity of the segmented (CSR) reductions: device-offset entry points
and plans, bitwise against the order model and within the rigorous bound."""
import numpy as np
import pytest
import torch

import oracle
import paper_1401_0248_amd as tf
import synth
from gpu_helpers import DEV, launch, same_bits, to_dev

pytestmark = pytest.mark.gpu


def _u(dtype):
    return 2.0 ** -(np.finfo(dtype).nmant + 1)


def _lengths():
    # empty, one element, exactly one tile, one past, many tiles, ragged
    return np.array([0, 1, 3, 256, 257, 1024, 1025, 5000, 0, 0, 77, 12345, 2, 65536 + 7, 0, 9],
                    dtype=np.int64)


def _rows(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("is_dot,mode", [(d, m) for d in (False, True)
                                         for m in ("plain", "fast", "rigorous", "kahan")]
                         + [(True, "fast_rounded"), (True, "rigorous_rounded")])
def test_seg_bitwise_vs_model(dtype, is_dot, mode):
    W = 16 // np.dtype(dtype).itemsize
    L = _lengths()
    off = synth.offsets_from_lengths(L)
    n = int(off[-1])
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(n) * np.exp2(rng.integers(-8, 8, n))).astype(dtype)
    y = rng.standard_normal(n).astype(dtype)
    for ts, u, gb, bt, xs, ys in ((64 * W, 1, 1, 64, 0, 0), (64 * W * 4, 4, 3, 256, 1, 0),
                                  (64 * W * 16, 8, 50, 512, 3, 3), (64 * W * 2, 2, 1000, 128, 2, 1)):
        xd, mis = to_dev(x, xs)
        yd, _ = to_dev(y, ys) if is_dot else (None, 0)
        od = torch.from_numpy(off).to(DEV)
        lc = launch(bt, u, gb, ts)
        got = tf.segdot(xd, yd, od, mode, lc) if is_dot else tf.segsum(xd, od, mode, lc)
        want = oracle.model_seg(mode, x, off, y if is_dot else None, mis, u, ts)
        g = _rows(got)
        for s in range(len(L)):
            assert same_bits(g[s], want[s]), (s, L[s], ts, u, gb, list(g[s]), list(want[s]))
        # the plan path gives the same bits
        plan = tf.SegPlan(off, xd.dtype, is_dot, mode, lc)
        got2 = plan.execute(xd, yd if is_dot else None)
        assert torch.equal(got2, got)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_seg_bound_default_launch(dtype):
    u = _u(dtype)
    L = synth.segment_lengths(3, 500, max_len=1 << 16)
    off = synth.offsets_from_lengths(L)
    x, y = synth.uniform(33, int(off[-1]), dtype, count=2)
    xd, _ = to_dev(x)
    yd, _ = to_dev(y)
    od = torch.from_numpy(off).to(DEV)
    gd = _rows(tf.segdot(xd, yd, od, "rigorous"))
    gs = _rows(tf.segsum(xd, od, "rigorous"))
    gf = _rows(tf.segsum(xd, od, "fast"))
    for s in range(0, len(L), 7):
        a, b = off[s], off[s + 1]
        ex = oracle.Exact(x[a:b], y[a:b])
        assert abs(ex.diff(*gd[s])) <= 4 * (b - a) * u * u * ex.A
        exs = oracle.Exact(x[a:b])
        assert exs.diff(*gs[s]) == 0.0 and exs.diff(*gf[s]) == 0.0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_wide_plan_vs_model(dtype):
    L = _lengths()
    off = synth.offsets_from_lengths(L)
    x, y = synth.uniform(4, int(off[-1]), dtype, count=2)
    xd, mis = to_dev(x, 1)
    yd, _ = to_dev(y, 0)
    W = 16 // np.dtype(dtype).itemsize
    ts = 64 * W * 4
    lc = launch(256, 4, 17, ts)
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    od = torch.from_numpy(np.asarray(off, dtype=np.int64)).to(DEV)
    for is_dot in (False, True):
        plan = tf.SegPlan(off, tdt, is_dot, "wide", lc)
        got = _rows(plan.execute(xd, yd if is_dot else None))
        want = oracle.model_seg("wide", x, off, y if is_dot else None, mis, 4, ts)
        for s in range(len(L)):
            assert same_bits(got[s], want[s]), s
        if dtype == np.float64:  # the device-offset path takes binary64 wide too
            dev = _rows(tf.segdot(xd, yd, od, "wide", lc) if is_dot else tf.segsum(xd, od, "wide", lc))
            for s in range(len(L)):
                assert same_bits(dev[s], want[s]), s
        # the typed device-offset calls (segsumd / segdotd), both data types
        got_d = tf.segdotd(xd, yd, od, lc) if is_dot else tf.segsumd(xd, od, lc)
        assert got_d.dtype == torch.float64
        dev = _rows(got_d)
        for s in range(len(L)):
            assert same_bits(dev[s], want[s]), s


@pytest.mark.parametrize("is_dot", [False, True])
def test_mixed_device_offsets_vs_model(is_dot):
    """The mixed form through the device-offset calls (segsum_mixed /
    segdot_mixed): bitwise the order model's and the plan's, binary64 rows."""
    L = _lengths()
    off = synth.offsets_from_lengths(L)
    n = int(off[-1])
    rng = np.random.default_rng(8)
    x = (rng.standard_normal(n) * np.exp2(rng.integers(-12, 12, n))).astype(np.float32)
    y = rng.standard_normal(n).astype(np.float32)
    od = torch.from_numpy(off).to(DEV)
    for ts, u, gb, bt, xs, ys in ((256, 1, 1, 64, 0, 0), (1024, 4, 3, 256, 1, 2),
                                  (4096, 8, 50, 512, 3, 3)):
        xd, mis = to_dev(x, xs)
        yd, _ = to_dev(y, ys)
        lc = launch(bt, u, gb, ts)
        got = tf.segdot_mixed(xd, yd, od, lc) if is_dot else tf.segsum_mixed(xd, od, lc)
        assert got.dtype == torch.float64
        want = oracle.model_seg("mixed", x, off, y if is_dot else None, mis, u, ts)
        g = _rows(got)
        for s in range(len(L)):
            assert same_bits(g[s], want[s]), (s, ts, u)
        plan = tf.SegPlan(off, torch.float32, is_dot, "mixed", lc)
        assert torch.equal(plan.execute(xd, yd if is_dot else None), got)
        plan.close()
    # default launch, and the checks of the typed calls
    got = tf.segdot_mixed(xd, yd, od) if is_dot else tf.segsum_mixed(xd, od)
    assert torch.isfinite(got).all()
    with pytest.raises(TypeError):
        tf.segsum_mixed(xd.double(), od)
    with pytest.raises(tf.TwofoldError):
        tf.segsum(xd, od, "mixed")


def test_invalid_device_offsets_give_nan():
    x = torch.ones(100, dtype=torch.float32, device=DEV)
    for bad in ([0, 50, 40, 100], [0, 50, 101], [-1, 5, 10]):
        od = torch.tensor(bad, dtype=torch.int64, device=DEV)
        out = _rows(tf.segsum(x, od, "rigorous"))
        assert np.all(np.isnan(out)), bad
    # a valid call on the same workspace afterwards is fine again
    od = torch.tensor([0, 50, 50, 100], dtype=torch.int64, device=DEV)
    out = _rows(tf.segsum(x, od, "rigorous"))
    assert list(out[:, 0]) == [50.0, 0.0, 50.0] and list(out[:, 1]) == [0.0, 0.0, 0.0]


def test_plan_graph_replay():
    L = synth.segment_lengths(7, 300, max_len=1 << 15)
    off = synth.offsets_from_lengths(L)
    x, y = synth.uniform(8, int(off[-1]), np.float64, count=2)
    xd, _ = to_dev(x)
    yd, _ = to_dev(y)
    plan = tf.SegPlan(off, torch.float64, True, "rigorous")
    eager = plan.execute(xd, yd).clone()
    out = torch.empty_like(eager)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ws = tf.workspace(plan.workspace_bytes, xd.device)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.execute(xd, yd, out=out, ws=ws)
    for i in range(5):
        out.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, eager), i
        plan.execute(yd, xd)
        torch.cuda.synchronize()
    for _ in range(20):
        assert torch.equal(plan.execute(xd, yd), eager)


def test_device_offset_calls_graph_replay():
    """Device-offset calls (tile table built on the device, then the tile and
    combine kernels) captured into a HIP graph: every replay, with other
    work between replays, equals the eager result bit for bit. Binary32 data
    in the mixed form and in sumd (binary64 rows), and a rigorous binary32
    dot (binary32 rows)."""
    L = synth.segment_lengths(9, 400, max_len=1 << 14)
    off = synth.offsets_from_lengths(L)
    x, y = synth.uniform(10, int(off[-1]), np.float32, count=2)
    xd, _ = to_dev(x, 1)
    yd, _ = to_dev(y, 1)
    od = torch.from_numpy(off).to(DEV)
    calls = [lambda o, w: tf.segdot_mixed(xd, yd, od, out=o, ws=w),
             lambda o, w: tf.segsumd(xd, od, out=o, ws=w),
             lambda o, w: tf.segdot(xd, yd, od, "rigorous", out=o, ws=w)]
    eager = [tf.segdot_mixed(xd, yd, od), tf.segsumd(xd, od), tf.segdot(xd, yd, od, "rigorous")]
    outs = [torch.empty_like(e) for e in eager]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        wss = [tf.Workspace(1 << 22, xd.device) for _ in calls]
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for c, o, w in zip(calls, outs, wss):
            c(o, w)
    for i in range(4):
        for o in outs:
            o.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for e, o in zip(eager, outs):
            assert torch.equal(o.view(torch.int8), e.view(torch.int8)), i
        tf.segdot_mixed(yd, xd, od)  # other work on the same tensors between replays
        torch.cuda.synchronize()


def test_plan_after_device_path_on_shared_workspace():
    """A device-offset call with few segments, then one with many, then a
    plan with many more, all on the same per-stream workspace: the plan's
    counters are its own, so earlier calls cannot disturb it."""
    W = 4
    for nseg_dev, nseg_plan in ((10, 3000), (3000, 10), (500, 500)):
        L = synth.segment_lengths(nseg_dev + nseg_plan, nseg_plan, max_len=1 << 13)
        off = synth.offsets_from_lengths(L)
        x = synth.uniform(1, int(off[-1]), np.float32)
        xd, mis = to_dev(x)
        Ld = synth.segment_lengths(nseg_dev, nseg_dev, max_len=1 << 13)
        offd = synth.offsets_from_lengths(Ld)
        xdev, _ = to_dev(synth.uniform(2, int(offd[-1]), np.float32))
        tf.segsum(xdev, torch.from_numpy(offd).to(DEV), "rigorous", launch(256, 4, 64, 64 * W))
        plan = tf.SegPlan(off, torch.float32, False, "rigorous", launch(256, 4, 64, 64 * W))
        got = _rows(plan.execute(xd))
        want = oracle.model_seg("rigorous", x, off, None, mis, 4, 64 * W)
        assert all(same_bits(got[s], want[s]) for s in range(len(L)))


def test_many_tiny_segments():
    L = np.ones(100000, dtype=np.int64)
    L[::3] = 0
    off = synth.offsets_from_lengths(L)
    x = synth.uniform(2, int(off[-1]), np.float32)
    xd, _ = to_dev(x)
    od = torch.from_numpy(off).to(DEV)
    got = _rows(tf.segsum(xd, od, "rigorous"))
    want = np.zeros(L.size)
    want[L == 1] = x
    assert np.array_equal(got[:, 0], want) and np.all(got[:, 1] == 0)


def _ragged_offsets(seed, nseg, max_len):
    rng = np.random.default_rng(seed)
    L = rng.integers(0, max_len + 1, nseg).astype(np.int64)
    L[rng.random(nseg) < 0.2] = 0
    return synth.offsets_from_lengths(L)


@pytest.mark.parametrize("nseg", [1023, 1024, 1025, 3073])
def test_device_offsets_across_rows_vs_model(nseg):
    """Segment counts around the tiling kernels' rows of 1024 segments, at a
    launch with a wave table and at one with more than 2^20 waves (no wave
    table: the tile kernel finds its bounds by search). Device-offset calls
    and plans, bitwise against the order model."""
    W = 4
    off = _ragged_offsets(nseg, nseg, 300)
    x = synth.uniform(nseg + 1, int(off[-1]), np.float32)
    xd, mis = to_dev(x, 1)
    od = torch.from_numpy(off).to(DEV)
    for bt, u, gb, ts in ((256, 2, 64, 64 * W * 2), (128, 1, (1 << 19) + 8, 64 * W)):
        lc = launch(bt, u, gb, ts)
        want = oracle.model_seg("rigorous", x, off, None, mis, u, ts)
        gt = tf.segsum(xd, od, "rigorous", lc)
        got = _rows(gt)
        bad = [s for s in range(nseg) if not same_bits(got[s], want[s])]
        assert not bad, (nseg, gb, bad[:5])
        plan = tf.SegPlan(off, xd.dtype, False, "rigorous", lc)
        assert torch.equal(plan.execute(xd).view(torch.int32), gt.view(torch.int32))
        plan.close()


def test_invalid_device_offsets_in_a_later_row():
    """An offset that decreases in the fourth row of 1024 segments, or a last
    offset past the data, makes every segment NaN; the same workspace then
    serves a valid call."""
    nseg = 5000
    off = _ragged_offsets(11, nseg, 40)
    x = torch.ones(int(off[-1]), dtype=torch.float32, device=DEV)
    ws = tf.Workspace(1 << 24, DEV)
    for s, delta in ((3500, -(int(off[3500] - off[3499]) + 1)), (nseg, 1)):
        bad = off.copy()
        bad[s] += delta
        assert bad[s] < bad[s - 1] or bad[-1] > off[-1]
        out = _rows(tf.segsum(x, torch.from_numpy(bad).to(DEV), "rigorous", ws=ws))
        assert np.all(np.isnan(out)), s
    out = _rows(tf.segsum(x, torch.from_numpy(off).to(DEV), "rigorous", ws=ws))
    assert np.array_equal(out[:, 0], np.diff(off).astype(np.float64)) and np.all(out[:, 1] == 0)


def test_more_rows_than_the_row_grid():
    """65,536 x 1024 + 1500 segments of 0, 1 or 2 small integers: the tiling
    kernels stride over more rows than they launch blocks, and the combine
    kernel over more segments than its grid. Every sum is exact."""
    nseg = 65536 * 1024 + 1500
    rng = np.random.default_rng(12)
    L = rng.integers(0, 3, nseg).astype(np.int64)
    off = synth.offsets_from_lengths(L)
    del L
    n = int(off[-1])
    xi = rng.integers(-8, 9, n).astype(np.int64)
    cs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(xi, out=cs[1:])
    want = (cs[off[1:]] - cs[off[:-1]]).astype(np.float64)
    del cs
    xd = torch.from_numpy(xi.astype(np.float32)).to(DEV)
    del xi
    od = torch.from_numpy(off).to(DEV)
    got = tf.segsum(xd, od, "rigorous").cpu().numpy().astype(np.float64)
    assert np.array_equal(got[:, 0], want)
    assert np.all(got[:, 1] == 0)
