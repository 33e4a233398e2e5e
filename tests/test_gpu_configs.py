"""GPU parity at the full sizes of the benchmark configurations.

* 2^20 binary64 uniform pairs (seed 0): rigorous sum and dot.
* Ill-conditioned dots, N = 2^24, binary32 and binary64, target conditions
  1e6 ... 1e16: the bench's workload, in the launch the bench times.
* 1 GiB per vector (roofline sweep sizes).
* Scaled binary32 dots, N = 2^26 (the precision study).
* 20,000 segments, lengths log-uniform in [1, 2^20] (1.5e9 elements):
  sampled segments.

Bitwise comparisons use explicit launch shapes written here. For the
bench's own launch the tuned table's values are restated below and
checked against the library, so the model's inputs never come from the
GPU path; a re-tuned table (which changes result bits) fails that check
until these constants are updated with it.
"""
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
import paper_1401_0248_amd as tf
from oracle import bounds
import synth
from gpu_helpers import DEV, pair, same_bits, to_dev

pytestmark = pytest.mark.gpu

N_ILL = 1 << 24
# (dtype, is_dot, mode) -> (block_threads, unroll, max_blocks) for 2^22 < n <= 2^24
BENCH_TABLE = {(8, 1, "rigorous"): (256, 2, 256), (8, 1, "fast"): (256, 4, 256),
               (4, 1, "rigorous"): (256, 2, 256), (4, 1, "fast"): (512, 1, 256)}
# segmented dots above 2^29 elements: (block_threads, unroll, grid, tile)
SEG_TABLE = {(4, "rigorous"): (256, 2, 256, 16384), (4, "fast"): (256, 2, 256, 32768),
             (8, "rigorous"): (256, 8, 256, 32768), (8, "fast"): (256, 8, 256, 32768)}


def _u(dtype):
    return 2.0 ** -(np.finfo(dtype).nmant + 1)


def _note(msg):
    print("[config] " + msg, file=sys.stderr, flush=True)


def _bench_launch(dtype, mode, n):
    """The launch the bench times, from this file's table; checked against
    the library's tuned default."""
    bt, u, maxb = BENCH_TABLE[(np.dtype(dtype).itemsize, 1, mode)]
    W = 16 // np.dtype(dtype).itemsize
    nv = (n + W - 1) // W
    gb = max(1, min(maxb, -(-nv // (bt * u))))
    lib = tf.default_launch(0, np.dtype(dtype).itemsize, True, mode, n)
    assert (lib.block_threads, lib.unroll, lib.grid_blocks) == (bt, u, gb), \
        "tuned table changed: update BENCH_TABLE (result bits depend on it)"
    return tf.Launch(bt, u, gb, 0, 0), (bt, u, gb)


def test_uniform_2e20_f64_seed0():
    n = 1 << 20
    x, y = synth.uniform(0, n, np.float64, count=2)
    xd, mis = to_dev(x)
    yd, _ = to_dev(y)
    u = _u(np.float64)
    ex = oracle.Exact(x, y)
    exs = oracle.Exact(x)
    for mode in ("rigorous", "fast", "plain"):
        v, e = pair(tf.sum(xd, mode))
        if mode != "plain":
            assert exs.diff(v, e) == 0.0, mode
        v, e = pair(tf.dot(xd, yd, mode))
        if mode == "rigorous":
            assert abs(ex.diff(v, e)) <= 4 * n * u * u * ex.A
    # bitwise against the model in an explicit launch
    lc = tf.Launch(512, 4, 64, 0, 0)
    got = pair(tf.dot(xd, yd, "rigorous", lc))
    assert same_bits(got, oracle.model_single("rigorous", x, y, mis, 512, 4, 64))


@pytest.fixture(scope="module")
def illcond():
    jobs = [(dt, d) for dt in (np.float32, np.float64) for d in (6, 8, 10, 12, 14, 16)]

    def one(job):
        dt, d = job
        return job, synth.illcond_dot(synth.illcond_seed(d), N_ILL, 10.0 ** d, dt)

    with ThreadPoolExecutor(max_workers=12) as ex:
        return dict(ex.map(one, jobs))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_illconditioned_bench_workload(illcond, dtype):
    u = _u(dtype)
    devs, singles = [], {}
    for d in (6, 8, 10, 12, 14, 16):
        x, y = illcond[(dtype, d)]
        _note("ill-conditioned %s cond 1e%d" % (np.dtype(dtype).name, d))
        xd, mis = to_dev(x)
        yd, _ = to_dev(y)
        devs.append((xd, yd))
        ex = oracle.Exact(x, y)
        for mode in ("rigorous", "fast"):
            lc, (bt, un, gb) = _bench_launch(dtype, mode, N_ILL)
            got_default = pair(tf.dot(xd, yd, mode))
            got = pair(tf.dot(xd, yd, mode, lc))
            assert same_bits(got, got_default)
            singles[(d, mode)] = got
            want, sv = oracle.model_single(mode, x, y, mis, bt, un, gb, with_violations=True)
            assert same_bits(got, want), (d, mode, got, list(want))
            # within the bound of the launch's own tree (the fast form's
            # widened by the steps that break Theorem 1's condition)
            assert abs(ex.diff(*got)) <= bounds.single_bound(dtype, N_ILL, bt, un, gb, ex.A, sv), \
                (d, mode, got)
            if mode == "rigorous":
                assert abs(ex.diff(*got)) <= 4 * N_ILL * u * u * ex.A, (d, got)
        if dtype == np.float32:
            # the mixed form of the same data, default launch: the order
            # model bit for bit and within the mixed tree bound
            dl = tf.default_launch(0, 4, True, "mixed", N_ILL)
            got = pair(tf.dot_mixed(xd, yd))
            want = oracle.model_single("mixed", x, y, mis, dl.block_threads, dl.unroll,
                                       dl.grid_blocks)
            assert same_bits(got, want), (d, got, list(want))
            Lc, D = bounds.single_depths(dtype, N_ILL, dl.block_threads, dl.unroll, dl.grid_blocks)
            assert abs(ex.diff(*got)) <= bounds.mixed_bound(Lc, D, ex.A), (d, got)
        if dtype == np.float64:
            # the wide accumulator (double-word) of the same data, default launch
            dl = tf.default_launch(0, 8, True, "wide", N_ILL)
            got = pair(tf.dotd(xd, yd))
            Lc, D = bounds.single_depths(dtype, N_ILL, dl.block_threads, dl.unroll, dl.grid_blocks)
            assert abs(ex.diff(*got)) <= bounds.dw_bound(Lc, D, ex.A), (d, got)
        # the plain value of the same launch is the twofold value
        lc, _ = _bench_launch(dtype, "rigorous", N_ILL)
        assert pair(tf.dot(xd, yd, "plain", lc))[0] == pair(tf.dot(xd, yd, "rigorous", lc))[0]
    # the bench's step: one multi-vector call per form over the six pairs,
    # default launch; every row is the single call's pair checked above
    for mode in ("rigorous", "fast"):
        out = tf.multidot([p[0] for p in devs], [p[1] for p in devs], mode)
        for i, d in enumerate((6, 8, 10, 12, 14, 16)):
            assert same_bits(pair(out[i]), singles[(d, mode)]), (mode, d)


def test_one_gib_sum_f32_exact_grid():
    n = 1 << 28
    _note("1 GiB binary32 sum")
    x = synth.uniform(1, n, np.float32)
    xd, mis = to_dev(x)
    ex = oracle.Exact(x)
    for mode in ("rigorous", "fast"):
        v, e = pair(tf.sum(xd, mode))
        assert ex.diff(v, e) == 0.0, mode
    lc = tf.Launch(256, 8, 256, 0, 0)
    got = pair(tf.sum(xd, "rigorous", lc))
    assert same_bits(got, oracle.model_single("rigorous", x, None, mis, 256, 8, 256))


def test_one_gib_dot_f64():
    n = 1 << 27
    _note("1 GiB binary64 dot")
    x, y = synth.uniform(1, n, np.float64, count=2)
    xd, mis = to_dev(x)
    yd, _ = to_dev(y)
    ex = oracle.Exact(x, y)
    u = _u(np.float64)
    v, e = pair(tf.dot(xd, yd, "rigorous"))
    assert abs(ex.diff(v, e)) <= 4 * n * u * u * ex.A
    lc = tf.default_launch(0, 8, True, "rigorous", n)
    assert abs(ex.diff(v, e)) <= bounds.single_bound(np.float64, n, lc.block_threads, lc.unroll,
                                                     lc.grid_blocks, ex.A)
    dl = tf.default_launch(0, 8, True, "wide", n)
    Lc, D = bounds.single_depths(np.float64, n, dl.block_threads, dl.unroll, dl.grid_blocks)
    assert abs(ex.diff(*pair(tf.dotd(xd, yd)))) <= bounds.dw_bound(Lc, D, ex.A)
    lc = tf.Launch(512, 2, 256, 0, 0)
    got = pair(tf.dot(xd, yd, "rigorous", lc))
    assert same_bits(got, oracle.model_single("rigorous", x, y, mis, 512, 2, 256))
    exs = oracle.Exact(x)
    assert exs.diff(*pair(tf.sum(xd, "rigorous"))) == 0.0


def test_scaled_f32_precision_study():
    """Binary32 twofold against binary64 plain (dotd) on the same binary32
    data: both within their bounds; the measured errors are reported."""
    n = 1 << 26
    _note("scaled binary32 dots, N=2^26")
    x, y = synth.scaled(2, n)
    xd, _ = to_dev(x)
    yd, _ = to_dev(y)
    ex = oracle.Exact(x, y)
    u32 = _u(np.float32)
    v, e = pair(tf.dot(xd, yd, "rigorous"))
    rig = abs(ex.diff(v, e))
    assert rig <= 4 * n * u32 * u32 * ex.A
    vd, ed = pair(tf.dotd(xd, yd))
    assert ed == 0.0
    wide = abs(ex.diff(vd))
    # binary64 accumulation of exact products: a tree of depth well below n
    assert wide <= n * 2.0 ** -53 * ex.A
    vf, ef = pair(tf.dot(xd, yd, "fast"))
    fast = abs(ex.diff(vf, ef))
    assert fast <= 4 * n * u32 * u32 * ex.A + 2 * u32 * ex.A
    _note("errors / sum|xy|: rigorous %.3g, fast %.3g, binary64 plain %.3g"
          % (rig / ex.A, fast / ex.A, wide / ex.A))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_segmented_full_batch_sampled(dtype):
    lengths = synth.segment_lengths(3, 20000)
    off = synth.offsets_from_lengths(lengths)
    n = int(off[-1])
    _note("segmented %s, %d elements" % (np.dtype(dtype).name, n))
    tdt = torch.float32 if dtype == np.float32 else torch.float64
    host = np.empty(2 * n, dtype=dtype)
    i = 0
    for c in synth.uniform_chunks(3, 2 * n, dtype):
        host[i:i + c.size] = c
        i += c.size
    x, y = host[:n], host[n:]
    both = torch.empty(2 * n, dtype=tdt, device=DEV)
    step = 1 << 26
    for a in range(0, 2 * n, step):
        both[a:a + step].copy_(torch.from_numpy(host[a:a + step]))
    xd, yd = both[:n], both[n:]
    W = 16 // np.dtype(dtype).itemsize
    mis = (xd.data_ptr() % 16) // np.dtype(dtype).itemsize
    size = np.dtype(dtype).itemsize
    lcs = {}
    for form in ("rigorous", "fast"):
        bt, un, gb, ts = SEG_TABLE[(size, form)]
        lib = tf.default_launch(1, size, True, form, n, len(lengths))
        assert (lib.block_threads, lib.unroll, lib.grid_blocks, lib.tile_elems) == (bt, un, gb, ts), \
            "tuned table changed: update SEG_TABLE (result bits depend on it)"
        lcs[form] = tf.Launch(bt, un, gb, 0, ts)
    got = tf.SegPlan(off, tdt, True, "rigorous", lcs["rigorous"]).execute(xd, yd).double().cpu().numpy()
    gotf = tf.SegPlan(off, tdt, True, "fast", lcs["fast"]).execute(xd, yd).double().cpu().numpy()
    dflt = tf.SegPlan(off, tdt, True, "rigorous").execute(xd, yd).double().cpu().numpy()
    assert np.array_equal(dflt.view(np.uint64), got.view(np.uint64))
    u = _u(dtype)
    rng = np.random.default_rng(0)
    sample = sorted(set(rng.integers(0, len(lengths), 30).tolist()) |
                    {int(np.argmax(lengths)), int(np.argmin(lengths))})
    for s in sample:
        a, b = int(off[s]), int(off[s + 1])
        xs, ys = x[a:b], y[a:b]
        smis = (mis + a) % W
        ex = oracle.Exact(xs, ys)
        assert abs(ex.diff(*got[s])) <= 4 * (b - a) * u * u * ex.A, s
        lr, lf = lcs["rigorous"], lcs["fast"]
        assert abs(ex.diff(*got[s])) <= bounds.segment_bound(dtype, b - a, lr.tile_elems, ex.A), s
        want = oracle.model_seg("rigorous", xs, [0, b - a], ys, smis, lr.unroll, lr.tile_elems)
        assert same_bits(got[s], want[0]), (s, b - a)
        wantf = oracle.model_seg("fast", xs, [0, b - a], ys, smis, lf.unroll, lf.tile_elems)
        assert same_bits(gotf[s], wantf[0]), (s, b - a)
    del both, host
    torch.cuda.empty_cache()


# binary32 sums above 2^31 elements: (block_threads, unroll, max_blocks) and
# the segmented (unroll, tile) of the tuned table, restated like the others
BIG_SUM = (256, 4, 256)
BIG_SEG_SUM = (8, 32768)


def test_beyond_2e31_elements():
    """A binary32 vector of 2^31 + 1027 elements (8 GiB): 64-bit indexing in
    the single-vector and segmented paths. Uniform data on the 2^-23 grid:
    v + e equals the exact sum, and every pair equals the order model's."""
    n = (1 << 31) + (1 << 10) + 3
    _note("2^31 + 1027 binary32 elements: generating")
    x = np.empty(n, dtype=np.float32)
    xd = torch.empty(n, dtype=torch.float32, device=DEV)
    i = 0
    for c in synth.uniform_chunks(21, n, np.float32, chunk=1 << 26):
        x[i:i + c.size] = c
        xd[i:i + c.size].copy_(torch.from_numpy(c))
        i += c.size
    mis = (xd.data_ptr() % 16) // 4
    bt, un, gb = BIG_SUM
    lib = tf.default_launch(0, 4, False, "rigorous", n)
    assert (lib.block_threads, lib.unroll, lib.grid_blocks) == (bt, un, gb), \
        "tuned table changed: update BIG_SUM (result bits depend on it)"
    ex = oracle.Exact(x)
    lc = tf.Launch(bt, un, gb, 0, 0)
    for mode in ("rigorous", "fast"):
        _note("2^31 + 1027: %s sum" % mode)
        got = pair(tf.sum(xd, mode, lc))
        assert ex.diff(*got) == 0.0, mode
        assert same_bits(got, oracle.model_single(mode, x, None, mis, bt, un, gb)), mode
    assert ex.diff(*pair(tf.sum(xd, "rigorous"))) == 0.0
    # three segments, the middle one across element 2^31
    off = np.array([0, (1 << 30) + 5, (1 << 31) + 7, n], dtype=np.int64)
    su, sts = BIG_SEG_SUM
    lib = tf.default_launch(1, 4, False, "rigorous", n, 3)
    assert (lib.unroll, lib.tile_elems) == (su, sts), \
        "tuned table changed: update BIG_SEG_SUM (result bits depend on it)"
    _note("2^31 + 1027: segmented sum")
    plan = tf.SegPlan(off, torch.float32, False, "rigorous")
    got = plan.execute(xd).double().cpu().numpy()
    want = oracle.model_seg("rigorous", x, off, None, mis, su, sts)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))
    for s in range(3):
        assert oracle.Exact(x[off[s]:off[s + 1]]).diff(*got[s]) == 0.0, s
    plan.close()
    del xd
    torch.cuda.empty_cache()


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_permuted_illconditioned(dtype):
    """The permuted variant of the ill-conditioned dot (cond 1e16, N = 2^20):
    the running sums no longer cancel in order. Rigorous, fast and wide
    results equal the order model's and lie within their tree bounds."""
    n = 1 << 20
    x, y = synth.illcond_dot(synth.illcond_seed(16), n, 1e16, dtype)
    x, y = synth.permute_pairs(synth.illcond_perm_seed(16), x, y)
    _note("permuted ill-conditioned %s" % np.dtype(dtype).name)
    xd, mis = to_dev(x)
    yd, _ = to_dev(y)
    ex = oracle.Exact(x, y)
    bt, un, gb = 256, 4, 128
    lc = tf.Launch(bt, un, gb, 0, 0)
    for mode in ("rigorous", "fast"):
        got = pair(tf.dot(xd, yd, mode, lc))
        want, sv = oracle.model_single(mode, x, y, mis, bt, un, gb, with_violations=True)
        assert same_bits(got, want), mode
        assert abs(ex.diff(*got)) <= bounds.single_bound(dtype, n, bt, un, gb, ex.A, sv), mode
    got = pair(tf.dotd(xd, yd, lc))
    assert same_bits(got, oracle.model_single("wide", x, y, mis, bt, un, gb))
    if dtype == np.float64:
        Lc, D = bounds.single_depths(dtype, n, bt, un, gb)
        assert abs(ex.diff(*got)) <= bounds.dw_bound(Lc, D, ex.A)
    else:
        assert abs(ex.diff(got[0])) <= n * 2.0 ** -53 * ex.A
