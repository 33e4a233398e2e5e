"""A second, independent statement of the documented reduction order, in
numpy, pinning the oracle's order model bit for bit on small inputs.

The order model (oracle/order_model.c) replays the GPU library's order
element by element in C. Here the same order is written another way:
every (lane, chain) accumulator is an entry of a numpy array, each element
step is one vectorised update of all lanes that take an element at that
point of the order, and the wave, block and grid combines are array
operations over lane indices. numpy's elementwise arithmetic is IEEE
binary32/binary64 with round to nearest and no contraction, so both
descriptions must give the same bits. Slips that only move an element to
another lane or chain, or change the combine tree, leave exact-grid sums
exact and bounded results bounded; this comparison catches them.

The exact product remainder of binary64 factors is Dekker's two-product
with Veltkamp's split (exact without overflow or underflow, which the data
here avoids); of binary32 factors, the binary64 product minus p.

The order (steps 1-8 of the library's public header): head elements on
lanes 0.. chain 0; rounds of U vectors per lane, vector k = q*U*L + u*L +
lane, component j on chain j; tail elements on lanes 0.. chain 0; chains
merged in order; xor butterflies 1, 2, ..., 32 in each wave; waves in order;
block pairs widened to binary64 and, with more than one block, strided over
256 lanes then combined the same way; finalize. Segmented: tiles of TS
elements, one 64-lane wave each, tile pairs strided over 64 lanes.
"""
import numpy as np
import pytest

import oracle

F32, F64 = np.float32, np.float64
ERRORLESS = ("plain", "wide")


def _two_product_rem(x, y, p):
    """x*y - p exactly, for binary64 arrays (Dekker, with Veltkamp's split
    by 2^27 + 1)."""
    def split(a):
        c = F64(134217729.0) * a
        hi = c - (c - a)
        return hi, a - hi
    xh, xl = split(x)
    yh, yl = split(y)
    return ((xh * yh - p) + xh * yl + xl * yh) + xl * yl


def _rem(x, y, p):
    if x.dtype == F32:
        return (x.astype(F64) * y.astype(F64) - p.astype(F64)).astype(F32)
    return _two_product_rem(x, y, p)


def _step(mode, dot, s, e, xv, yv):
    """One element into each of the given chains (arrays), as the paper's
    steps state it; returns the new (s, e)."""
    if mode == "wide":
        item = xv.astype(F64) * yv.astype(F64) if dot else xv.astype(F64)
        return s + item, e
    if mode == "mixed":
        sv = s.astype(F32)
        p = xv * yv if dot else xv
        t = sv + p
        yt = t - sv
        dy = p - yt
        ds = sv - (t - yt)
        r = (ds + dy).astype(F64)
        if dot:
            r = r + _rem(xv, yv, p).astype(F64)
        return t.astype(F64), e + r
    p = xv * yv if dot else xv
    if mode == "plain":
        return s + p, e
    if mode == "kahan":
        yk = p + e
        t = s + yk
        return t, yk - (t - s)
    track = dot and mode in ("fast", "rigorous")
    t = s + p
    if mode in ("fast", "fast_rounded"):
        c = (t - s) - p
        return t, (e + (_rem(xv, yv, p) - c)) if track else e - c
    yt = t - s
    dy = p - yt
    ds = s - (t - yt)
    return t, (e + ((ds + dy) + _rem(xv, yv, p))) if track else e + (ds + dy)


def _combine(mode, s1, e1, s2, e2):
    """Pair combine: two-sum of the values (in binary32 for the mixed form),
    errors added, then the two-sum remainder."""
    if mode in ERRORLESS:
        return s1 + s2, np.zeros_like(e1)
    if mode == "mixed":
        a, b = s1.astype(F32), s2.astype(F32)
    else:
        a, b = s1, s2
    x = a + b
    bp = x - a
    ap = x - bp
    y = (a - ap) + (b - bp)
    if mode == "mixed":
        return x.astype(F64), (e1 + e2) + y.astype(F64)
    return x, (e1 + e2) + y


def _lanes(mode, dot, x, y, head, L, U, A):
    """Steps 1-4 over x (and y): (L,) arrays of each lane's merged pair."""
    W = 16 // x.itemsize
    n = x.size
    s = np.zeros((L, W), dtype=A)
    e = np.zeros((L, W), dtype=A)
    yy = y if dot else np.zeros_like(x)

    def put(lanes, chain, idx):
        s[lanes, chain], e[lanes, chain] = _step(mode, dot, s[lanes, chain], e[lanes, chain],
                                                 x[idx], yy[idx])

    if head:
        put(np.arange(head), 0, np.arange(head))
    V = (n - head) // W
    per_round = U * L
    for q in range((V + per_round - 1) // per_round):
        for u in range(U):
            k = q * per_round + u * L + np.arange(L)
            ok = k < V
            for j in range(W):
                put(np.nonzero(ok)[0], j, head + k[ok] * W + j)
    r = n - head - V * W
    if r:
        put(np.arange(r), 0, head + V * W + np.arange(r))
    ps, pe = s[:, 0].copy(), e[:, 0].copy()
    for j in range(1, W):
        ps, pe = _combine(mode, ps, pe, s[:, j], e[:, j])
    return ps, pe


def _waves(mode, s, e):
    """Step 5 on (..., 64) arrays: lane l combines with lane l ^ d, for
    d = 1, 2, ..., 32, on the pairs as they were before the step."""
    lane = np.arange(64)
    for d in (1, 2, 4, 8, 16, 32):
        s, e = _combine(mode, s, e, s[..., lane ^ d], e[..., lane ^ d])
    return s[..., 0], e[..., 0]


def _grid64(mode, ps, pe, nlanes):
    """Binary64 combine of the pairs over nlanes lanes: lane l folds pairs l,
    l + nlanes, ... in order from +0, then waves, then waves in order."""
    m = "rigorous" if mode == "mixed" else mode
    s = np.zeros(nlanes)
    e = np.zeros(nlanes)
    for i0 in range(0, ps.size, nlanes):
        c = min(nlanes, ps.size - i0)
        s[:c], e[:c] = _combine(m, s[:c], e[:c], ps[i0:i0 + c], pe[i0:i0 + c])
    ws, we = _waves(m, s.reshape(-1, 64), e.reshape(-1, 64))
    V, E = ws[:1], we[:1]
    for w in range(1, ws.size):
        V, E = _combine(m, V, E, ws[w:w + 1], we[w:w + 1])
    return float(V[0]), float(E[0])


def _finalize(mode, dtype, V, E):
    if dtype == F64 or mode == "wide":
        return V, E
    v = float(F32(V))
    if mode == "mixed":
        return v, (V - v) + E
    if mode in ERRORLESS:
        return v, 0.0
    return v, float(F32(F64(V - v) + F64(E)))


def _acc(mode, dtype):
    return F64 if mode in ("wide", "mixed") else dtype


def order_single(mode, x, y, mis, bt, U, gb):
    dot = y is not None
    W = 16 // x.itemsize
    head = min((W - mis % W) % W, x.size)
    ps, pe = _lanes(mode, dot, x, y, head, gb * bt, U, _acc(mode, x.dtype.type))
    ws, we = _waves(mode, ps.reshape(gb, bt // 64, 64), pe.reshape(gb, bt // 64, 64))
    bs, be = ws[:, 0], we[:, 0]
    for w in range(1, bt // 64):
        bs, be = _combine(mode, bs, be, ws[:, w], we[:, w])
    bs, be = bs.astype(F64), be.astype(F64)
    if gb == 1:
        V, E = float(bs[0]), float(be[0])
    else:
        V, E = _grid64(mode, bs, be, 256)
    return _finalize(mode, x.dtype.type, V, E)


def order_seg(mode, x, off, y, mis, U, TS):
    dot = y is not None
    W = 16 // x.itemsize
    out = []
    for sg in range(len(off) - 1):
        o0, o1 = int(off[sg]), int(off[sg + 1])
        ts, te = [], []
        for a in range(o0, o1, TS):
            b = min(o1, a + TS)
            head = min((W - (mis + a) % W) % W, b - a)
            ps, pe = _lanes(mode, dot, x[a:b], y[a:b] if dot else None, head, 64, U,
                            _acc(mode, x.dtype.type))
            s, e = _waves(mode, ps, pe)
            ts.append(float(s))
            te.append(float(e))
        if not ts:
            out.append((0.0, 0.0))
        elif len(ts) == 1:
            out.append(_finalize(mode, x.dtype.type, ts[0], te[0]))
        else:
            V, E = _grid64(mode, np.array(ts), np.array(te), 64)
            out.append(_finalize(mode, x.dtype.type, V, E))
    return np.array(out, dtype=F64).reshape(-1, 2)


FORMS = [(m, d) for m in ("plain", "fast", "rigorous", "kahan") for d in (False, True)] + \
        [("fast_rounded", True), ("rigorous_rounded", True)]
LAUNCHES = [(64, 1, 1), (128, 2, 3), (64, 4, 2), (256, 1, 5), (64, 2, 257), (64, 1, 300)]


def _data(rng, n, dtype):
    v = rng.standard_normal(n) * np.exp2(rng.integers(-20, 20, n))
    return v.astype(dtype)


def _bits(a):
    return np.asarray(a, dtype=F64).view(np.uint64)


@pytest.mark.parametrize("dtype", [F32, F64])
@pytest.mark.parametrize("launch", LAUNCHES)
def test_single_order_matches_the_model(dtype, launch):
    bt, U, gb = launch
    rng = np.random.default_rng(bt * 1000 + U * 10 + gb)
    W = 16 // np.dtype(dtype).itemsize
    forms = FORMS + ([("wide", False), ("wide", True), ("mixed", False), ("mixed", True)]
                     if dtype == F32 else [])
    for n in (0, 1, W + 1, 1000, bt * gb * W * U + 2 * W + 3, 3 * bt * gb * W * U + 1):
        x, y = _data(rng, n, dtype), _data(rng, n, dtype)
        for mode, dot in forms:
            mis = int(rng.integers(0, W))
            yy = y if dot else None
            want = oracle.model_single(mode, x, yy, mis, bt, U, gb)
            got = order_single(mode, x, yy, mis, bt, U, gb)
            assert np.array_equal(_bits(got), _bits(want)), (mode, dot, n, mis, got, list(want))


@pytest.mark.parametrize("dtype", [F32, F64])
def test_segmented_order_matches_the_model(dtype):
    rng = np.random.default_rng(11)
    W = 16 // np.dtype(dtype).itemsize
    TS = 64 * W
    lengths = [0, 1, 3, TS - 1, TS, TS + 1, 5 * TS + 7, 70 * TS + 5, 0, 2 * TS]
    off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
    x, y = _data(rng, int(off[-1]), dtype), _data(rng, int(off[-1]), dtype)
    forms = FORMS + ([("wide", True), ("mixed", False), ("mixed", True)] if dtype == F32 else [])
    for mode, dot in forms:
        for U, mis in ((1, 0), (2, W - 1), (4, 1 % W)):
            yy = y if dot else None
            want = oracle.model_seg(mode, x, off, yy, mis, U, TS)
            got = order_seg(mode, x, off, yy, mis, U, TS)
            assert np.array_equal(_bits(got), _bits(want)), (mode, dot, U, mis)


def test_two_product_remainder_is_exact():
    """Dekker's two-product against exact rational arithmetic."""
    from fractions import Fraction
    rng = np.random.default_rng(3)
    x = rng.standard_normal(2000) * np.exp2(rng.integers(-200, 200, 2000))
    y = rng.standard_normal(2000) * np.exp2(rng.integers(-200, 200, 2000))
    p = x * y
    r = _two_product_rem(x, y, p)
    for i in range(0, 2000, 7):
        assert Fraction(float(r[i])) == Fraction(float(x[i])) * Fraction(float(y[i])) - \
            Fraction(float(p[i]))
