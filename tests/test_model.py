"""Pins of the oracle's order model (the paper's steps applied in the GPU
library's documented reduction order).

* With the data confined to one lane's chain, the model must equal the
  paper's sequential loop bitwise (every other chain, lane, wave and block
  contributes (+0, +0), and combining with a zero pair is exact).
* Combines are exact (Theorem 2): on exact-grid data value + error equals
  the exact sum for every launch shape and both forms.
* Rigorous results satisfy |v + e - S| <= 4 N u^2 sum|x y|.
* The twofold value equals the plain value of the same order.
* A one-tile segment is a single-vector reduction with one 64-lane block.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
import synth

LAUNCHES = [(256, 1, 1), (256, 4, 3), (512, 2, 2), (1024, 8, 5), (64, 1, 1), (128, 2, 7)]


def _u(dtype):
    return 2.0 ** -(np.finfo(dtype).nmant + 1)


SEQ = {("plain", False): "sum", ("plain", True): "dot", ("fast", False): "sumtf",
       ("fast", True): "dottf", ("rigorous", False): "sumt", ("rigorous", True): "dott",
       ("kahan", False): "sumk_pair", ("kahan", True): "dotk_pair",
       ("fast_rounded", True): "dottf_rounded", ("rigorous_rounded", True): "dott_rounded"}


def _seq_kind(mode, is_dot):
    return SEQ[(mode, is_dot)]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("mode,is_dot", [(m, d) for (m, d) in SEQ])
def test_single_lane_reduces_to_sequential(dtype, mode, is_dot):
    W = 16 // np.dtype(dtype).itemsize
    bt, U, gb = 256, 2, 3
    L = bt * gb
    rng = np.random.default_rng(21)
    for mis in range(W):
        head = (W - mis) % W
        nvec = 37 * U * L + 5  # several rounds and a partial one
        n = head + nvec * W + (W - 1 if W > 1 else 0)
        r = n - head - nvec * W
        # lane 0, chain 0: head element 0 (if any), vectors k = q*U*L + u*L,
        # tail element 0 (if any)
        idx = []
        if head:
            idx.append(0)
        for k in range(0, nvec, L):
            idx.append(head + k * W)
        if r:
            idx.append(head + nvec * W)
        x = np.zeros(n, dtype=dtype)
        vals = (rng.standard_normal(len(idx)) * np.exp2(rng.integers(-8, 8, len(idx)))).astype(dtype)
        x[idx] = vals
        y = None
        yv = None
        if is_dot:
            y = rng.standard_normal(n).astype(dtype)
            yv = y[idx]
        got = oracle.model_single(mode, x, y, x_misalign=mis, block_threads=bt, unroll=U,
                                  grid_blocks=gb)
        v, e = oracle.seq(_seq_kind(mode, is_dot), vals, yv)
        assert got[0] == float(v) and got[1] == float(e), (mis, got, v, e)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("mode", ["fast", "rigorous"])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_exact_grid_all_launches(dtype, mode, launch):
    bt, U, gb = launch
    for n in (0, 1, 7, 1000, 65536 + 3):
        x = synth.uniform(n + 17, n, dtype)
        ex = oracle.Exact(x)
        for mis in (0, 16 // np.dtype(dtype).itemsize - 1):
            got = oracle.model_single(mode, x, None, mis, bt, U, gb)
            assert ex.diff(got[0], got[1]) == 0.0, (n, mis, got)
            plain = oracle.model_single("plain", x, None, mis, bt, U, gb)
            assert plain[0] == got[0] and plain[1] == 0.0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_rigorous_dot_bound_all_launches(dtype, launch):
    bt, U, gb = launch
    u = _u(dtype)
    for seed, n in ((1, 4099), (2, 1 << 16)):
        x, y = synth.uniform(seed, n, dtype, count=2)
        ex = oracle.Exact(x, y)
        got = oracle.model_single("rigorous", x, y, 0, bt, U, gb)
        assert abs(ex.diff(got[0], got[1])) <= 4 * n * u * u * ex.A
        plain = oracle.model_single("plain", x, y, 0, bt, U, gb)
        assert plain[0] == got[0]
        fast = oracle.model_single("fast", x, y, 0, bt, U, gb)
        assert fast[0] == got[0]


def test_illconditioned_rigorous_bound_model():
    for dtype in (np.float32, np.float64):
        u = _u(dtype)
        x, y = synth.illcond_dot(synth.illcond_seed(16), 1 << 16, 1e16, dtype)
        ex = oracle.Exact(x, y)
        got = oracle.model_single("rigorous", x, y, 0, 256, 4, 16)
        assert abs(ex.diff(got[0], got[1])) <= 4 * x.size * u * u * ex.A


def test_two_lanes_combine_exact():
    """Data only on lanes 0 and 1 (chain 0, first vector each): the result is
    the exact combine of two one-element chains."""
    rng = np.random.default_rng(5)
    for _ in range(200):
        a, b = rng.standard_normal(2) * np.exp2(rng.integers(-30, 30, 2))
        x = np.zeros(2 * 256 * 2, dtype=np.float64)
        x[0], x[2] = a, b  # vector 0 -> lane 0, vector 1 -> lane 1
        got = oracle.model_single("rigorous", x, None, 0, 256, 1, 1)
        assert F(got[0]) + F(got[1]) == F(a) + F(b)
        assert got[0] == a + b


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_tiny_sizes(dtype):
    assert list(oracle.model_single("rigorous", np.zeros(0, dtype))) == [0.0, 0.0]
    x = np.array([0.3], dtype=dtype)
    y = np.array([-0.7], dtype=dtype)
    got = oracle.model_single("rigorous", x)
    assert got[0] == float(x[0]) and got[1] == 0.0
    got = oracle.model_single("rigorous", x, y)
    p = (x * y)[0]
    assert got[0] == float(p)
    assert F(got[0]) + F(got[1]) == F(float(x[0])) * F(float(y[0]))


def test_wide_mode_matches_binary64_sum_of_widened():
    x, y = synth.uniform(8, 10000, np.float32, count=2)
    got = oracle.model_single("wide", x, None, 0, 256, 1, 1)
    ex = oracle.Exact(x)
    # binary64 sums of binary32 values with |x| < 1 and n < 2^29 are exact
    assert got[0] == ex.S and got[1] == 0.0
    got = oracle.model_single("wide", x, y, 0, 256, 1, 1)
    assert abs(got[0] - oracle.Exact(x, y).S) <= 1e-13


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("mode", ["plain", "fast", "rigorous"])
def test_one_tile_segment_is_single_block_of_64(dtype, mode):
    W = 16 // np.dtype(dtype).itemsize
    ts = 64 * W * 8
    rng = np.random.default_rng(3)
    for n in (1, 5, ts - 1, ts):
        for mis in range(W):
            x = rng.standard_normal(n).astype(dtype)
            y = rng.standard_normal(n).astype(dtype)
            seg = oracle.model_seg(mode, x, [0, n], y, x_misalign=mis, unroll=2, tile_elems=ts)
            one = oracle.model_single(mode, x, y, mis, 64, 2, 1)
            assert seg[0][0] == one[0] and seg[0][1] == one[1]


def test_segments_are_independent():
    rng = np.random.default_rng(9)
    lengths = [0, 1, 300, 1024, 1025, 5000, 0, 77]
    off = synth.offsets_from_lengths(lengths)
    x = rng.standard_normal(off[-1])
    y = rng.standard_normal(off[-1])
    ts = 1024
    allseg = oracle.model_seg("rigorous", x, off, y, 0, 4, ts)
    for s in range(len(lengths)):
        a, b = off[s], off[s + 1]
        # the segment alone, at the same alignment (a mod 2 elements)
        one = oracle.model_seg("rigorous", x[a:b], [0, b - a], y[a:b], int(a % 2), 4, ts)
        assert allseg[s][0] == one[0][0] and allseg[s][1] == one[0][1]
    assert list(allseg[0]) == [0.0, 0.0] and list(allseg[6]) == [0.0, 0.0]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_segmented_exact_grid_and_bound(dtype):
    W = 16 // np.dtype(dtype).itemsize
    ts = 64 * W * 4
    lengths = synth.segment_lengths(3, 60, max_len=1 << 14)
    off = synth.offsets_from_lengths(lengths)
    x, y = synth.uniform(31, int(off[-1]), dtype, count=2)
    got = oracle.model_seg("rigorous", x, off, None, 0, 4, ts)
    gotd = oracle.model_seg("rigorous", x, off, y, 0, 4, ts)
    u = _u(dtype)
    for s in range(len(lengths)):
        a, b = off[s], off[s + 1]
        assert oracle.Exact(x[a:b]).diff(*got[s]) == 0.0
        ex = oracle.Exact(x[a:b], y[a:b])
        assert abs(ex.diff(*gotd[s])) <= 4 * (b - a) * u * u * ex.A


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_kahan_and_rounded_forms(dtype):
    """Kahan's value is compensated: within the classical (2u + O(n u^2))
    sum|x| of the exact sum, far better than the plain value; its error is
    the pending correction. The rounded-product dots share the FMA dots'
    value but miss the products' rounding."""
    u = _u(dtype)
    x, y = synth.uniform(44, 1 << 15, dtype, count=2)
    ex = oracle.Exact(x)
    k = oracle.model_single("kahan", x, None, 1, 256, 2, 3)
    assert abs(ex.diff(k[0])) <= 2 * u * ex.A + 4 * x.size * u * u * ex.A
    assert abs(ex.diff(k[0], k[1])) <= abs(ex.diff(k[0]))
    exd = oracle.Exact(x, y)
    fr = oracle.model_single("rigorous_rounded", x, y, 0, 256, 2, 3)
    fm = oracle.model_single("rigorous", x, y, 0, 256, 2, 3)
    assert fr[0] == fm[0]
    assert abs(exd.diff(*fr)) > 10 * abs(exd.diff(*fm))


def test_model_rejects_bad_arguments():
    x = np.zeros(10)
    with pytest.raises(ValueError):
        oracle.model_single("rigorous", x, None, 0, 100, 1, 1)
    with pytest.raises(ValueError):
        oracle.model_single(9, x, None, 0, 256, 1, 1)
    with pytest.raises(ValueError):
        oracle.model_single("fast_rounded", x, None, 0, 256, 1, 1)
    with pytest.raises(ValueError):
        oracle.model_seg("rigorous", x, [0, 5, 3], None, 0, 1, 128)
    with pytest.raises(ValueError):
        oracle.model_seg("rigorous", x, [0, 10], None, 0, 1, 100)


# ---- launch-specific error bounds (oracle.bounds) ----------------------------
from oracle import bounds  # noqa: E402


_DATA = {}


def _datasets(dtype, n, seed):
    key = (np.dtype(dtype).name, n, seed)
    if key not in _DATA:
        sets = [("uniform",) + tuple(synth.uniform(seed, n, dtype, count=2)),
                ("illcond",) + tuple(synth.illcond_dot(synth.illcond_seed(16), n, 1e16, dtype))]
        if dtype == np.float32:
            sets.append(("scaled",) + tuple(synth.scaled(seed, n)))
        _DATA[key] = sets
    return _DATA[key]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_rigorous_within_tree_bound(dtype, launch):
    """The rigorous model result lies within the bound of its own tree, for
    sums and dots, on uniform, ill-conditioned and scaled data."""
    bt, U, gb = launch
    n = 1 << 14
    for name, x, y in _datasets(dtype, n, 7):
        for yy in (None, y):
            ex = oracle.Exact(x, yy)
            got = oracle.model_single("rigorous", x, yy, 1, bt, U, gb)
            b = bounds.single_bound(dtype, n, bt, U, gb, ex.A)
            assert abs(ex.diff(got[0], got[1])) <= b, (name, yy is None)
            assert b <= 4 * n * bounds.unit_roundoff(dtype) ** 2 * ex.A or gb * bt < 256


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_fast_within_violation_bound(dtype, launch):
    """The fast model result lies within the tree bound widened by the loss
    of the steps that break Theorem 1's condition, as the model counts them;
    the rigorous form counts none."""
    bt, U, gb = launch
    n = 1 << 14
    for name, x, y in _datasets(dtype, n, 8):
        for yy in (None, y):
            ex = oracle.Exact(x, yy)
            got, sv = oracle.model_single("fast", x, yy, 0, bt, U, gb, with_violations=True)
            b = bounds.single_bound(dtype, n, bt, U, gb, ex.A, fast_violations=sv)
            assert abs(ex.diff(got[0], got[1])) <= b, (name, yy is None, sv)
            _, sv_rig = oracle.model_single("rigorous", x, yy, 0, bt, U, gb, with_violations=True)
            assert sv_rig == 0.0


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_fast_equals_rigorous_without_violations(dtype):
    """Where no chain step breaks Theorem 1's condition, fast-two-sum's
    round-off is exact, so the fast pair equals the rigorous pair bit for
    bit. Positive items of decreasing size along every chain give such data;
    random signs give violations, and then the pairs may differ only in e."""
    n = 1 << 13
    rng = np.random.default_rng(12)
    x = (np.exp2(-np.arange(n) / 64.0) * (1 + rng.random(n))).astype(dtype)
    y = np.ones(n, dtype=dtype)
    for yy in (None, y):
        f, sv = oracle.model_single("fast", x, yy, 0, 256, 2, 2, with_violations=True)
        r = oracle.model_single("rigorous", x, yy, 0, 256, 2, 2)
        assert sv == 0.0
        assert f[0] == r[0] and f[1] == r[1]
    z = rng.standard_normal(n).astype(dtype)
    f, sv = oracle.model_single("fast", z, None, 0, 256, 2, 2, with_violations=True)
    r = oracle.model_single("rigorous", z, None, 0, 256, 2, 2)
    assert sv > 0.0 and f[0] == r[0]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_segments_within_tile_bound(dtype):
    W = 16 // np.dtype(dtype).itemsize
    ts = 64 * W * 4
    lengths = synth.segment_lengths(5, 80, max_len=1 << 14)
    off = synth.offsets_from_lengths(lengths)
    x, y = synth.illcond_dot(synth.illcond_seed(12), int(off[-1]), 1e12, dtype)
    for mode in ("rigorous", "fast"):
        got, sv = oracle.model_seg(mode, x, off, y, 0, 4, ts, with_violations=True)
        for s in range(len(lengths)):
            a, b = off[s], off[s + 1]
            ex = oracle.Exact(x[a:b], y[a:b])
            bd = bounds.segment_bound(dtype, b - a, ts, ex.A, fast_violations=sv[s])
            assert abs(ex.diff(*got[s])) <= bd, (mode, s)


def test_tree_bound_depths():
    """Depth bookkeeping on hand-counted launches."""
    # binary64, 1 block of 64 lanes, n = 64*2*10 elements: 10 vectors per
    # lane (+2 for head and tail); combines: 1 chain merge + 6 wave levels
    assert bounds.single_depths(np.float64, 1280, 64, 1, 1) == (11 + 2, 7)
    # binary32, 4 blocks of 256: + 3 block levels, + 1 strided + 6 + 3 in pass 2
    Lc, D = bounds.single_depths(np.float32, 4096 * 4, 256, 4, 4)
    assert D == 3 + 6 + 3 + 1 + 6 + 3
    assert Lc == -(-(4096 + 1) // 1024) + 2
    # a segment of three tiles: 3 + 6 inside the tile, 1 + 6 across tiles
    assert bounds.segment_depths(np.float32, 3 * 1024, 1024) == (-(-257 // 64) + 2, 3 + 6 + 1 + 6)


# ---- the wide accumulator (sumd/dotd): binary64 for binary32 data, double-
# ---- word for binary64 data ---------------------------------------------------
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("is_dot", [False, True])
def test_wide_single_lane_reduces_to_sequential(dtype, is_dot):
    """Data on one lane's chain: the model equals the sequential wide loop
    (sumd/dotd for binary32 data; the double-word sumdd/dotdd for binary64)."""
    W = 16 // np.dtype(dtype).itemsize
    bt, U, gb = 128, 2, 3
    L = bt * gb
    rng = np.random.default_rng(22)
    nvec = 11 * U * L + 7
    n = nvec * W
    idx = list(range(0, nvec, L))
    idx = [k * W for k in idx]
    x = np.zeros(n, dtype=dtype)
    vals = (rng.standard_normal(len(idx)) * np.exp2(rng.integers(-30, 30, len(idx)))).astype(dtype)
    x[idx] = vals
    y = rng.standard_normal(n).astype(dtype) if is_dot else None
    yv = y[idx] if is_dot else None
    got = oracle.model_single("wide", x, y, 0, bt, U, gb)
    if dtype == np.float64:
        v, e = oracle.seq("dotdd" if is_dot else "sumdd", vals, yv)
    else:
        v, e = oracle.seq("dotd" if is_dot else "sumd", vals, yv)
    assert got[0] == float(v) and got[1] == float(e)


@pytest.mark.parametrize("launch", LAUNCHES)
def test_double_word_within_bound(launch):
    """Binary64 wide results lie within the double-word bound of their tree
    and are normalized double-word numbers."""
    bt, U, gb = launch
    n = 1 << 14
    for name, x, y in _datasets(np.float64, n, 7):
        for yy in (None, y):
            ex = oracle.Exact(x, yy)
            got = oracle.model_single("wide", x, yy, 0, bt, U, gb)
            Lc, D = bounds.single_depths(np.float64, n, bt, U, gb)
            assert abs(ex.diff(got[0], got[1])) <= bounds.dw_bound(Lc, D, ex.A), (name, yy is None)
            assert got[0] == got[0] + got[1]  # normalized double-word result


def test_sequential_double_word_pinned_by_fractions():
    """The sequential double-word dot on small inputs: error at most
    (3u^2 + 13u^3) times the sum of the exact partial results' magnitudes."""
    u = 2.0 ** -53
    rng = np.random.default_rng(23)
    for trial in range(40):
        n = int(rng.integers(2, 200))
        x = rng.standard_normal(n) * np.exp2(rng.integers(-20, 20, n))
        y = rng.standard_normal(n) * np.exp2(rng.integers(-20, 20, n))
        if trial % 2:
            y[n // 2:] = -x[:n - n // 2] * y[:n - n // 2] / np.where(x[n // 2:] == 0, 1, x[n // 2:])
        v, e = oracle.seq("dotdd", x, y)
        part, tot = F(0), F(0)
        for a, b in zip(x, y):
            part += F(float(a)) * F(float(b))
            tot += abs(part)
        err = abs(F(float(v)) + F(float(e)) - part)
        assert err <= (F(3 * u * u) + 13 * F(u) ** 3) * tot * (1 + F(1, 1 << 20))


def test_double_word_segments_within_bound():
    ts = 64 * 2 * 4
    lengths = synth.segment_lengths(5, 80, max_len=1 << 14)
    off = synth.offsets_from_lengths(lengths)
    x, y = synth.illcond_dot(synth.illcond_seed(12), int(off[-1]), 1e12, np.float64)
    got = oracle.model_seg("wide", x, off, y, 0, 4, ts)
    for s in range(len(lengths)):
        a, b = off[s], off[s + 1]
        ex = oracle.Exact(x[a:b], y[a:b])
        Lc, D = bounds.segment_depths(np.float64, b - a, ts)
        assert abs(ex.diff(*got[s])) <= bounds.dw_bound(Lc, D, ex.A), s
