"""The error bounds of oracle/bounds.py, pinned from both sides.

From below (a bound must hold): every result of the searches here lies
within its bound. From above (a bound must not be loose by orders of
magnitude): seeded searches over inputs built to make the roundings large
reach a stated fraction of each bound, so a bound that is far too loose
(a u where u^2 belongs, a dropped factor u) fails, and so does one that is
far too tight (a dropped loss term, a bound scaled down).

The searches run the oracle's own statements of the methods (the
sequential paper loops, the double-word additions, the order model of the
GPU tree) and measure |v + e - S| exactly (Fraction or the exact
accumulator). The fractions asserted are what the seeded searches reach,
rounded down: the fast form's loss term is reached almost exactly; a
double-word addition reaches a third of its per-operation bound; a
three-item rigorous chain a fortieth; a GPU-order tree of a few hundred
items about 1/200.
"""
from fractions import Fraction as F

import numpy as np
import pytest

import oracle
from oracle import bounds

DTYPES = [np.float32, np.float64]


def _err(v, e, terms):
    S = sum((F(float(t)) for t in terms), F(0))
    return abs(F(float(v)) + F(float(e)) - S)


@pytest.mark.parametrize("dtype", DTYPES)
def test_fast_loss_term_is_reached(dtype):
    """One step that breaks Theorem 1's condition (|running sum| < |item|):
    the fast form's error approaches u (1 + 2u) |item|, the loss the bound
    allows for it, and never exceeds the bound."""
    rng = np.random.default_rng(3)
    worst = 0.0
    for _ in range(4000):
        b = dtype(rng.uniform(0.5, 1) * (1 if rng.random() < 0.5 else -1))
        a = dtype(rng.uniform(-1, 1) * 2.0 ** -int(rng.integers(1, 30)))
        xs = np.array([a, b], dtype=dtype)
        v, e = oracle.seq("sumtf", xs)
        bd = bounds.tree_bound(dtype, 2, 0, abs(float(a)) + abs(float(b)),
                               fast_violations=abs(float(b)))
        r = float(_err(v, e, xs)) / bd
        assert r <= 1.0, (a, b, r)
        worst = max(worst, r)
    assert worst > 0.95, worst


@pytest.mark.parametrize("dtype", DTYPES)
def test_rigorous_chain_bound_is_approached(dtype):
    """Three-item rigorous chains (Example 3 in sequence): the error term's
    own rounding reaches 1/40 of the tree bound of a chain of three."""
    rng = np.random.default_rng(1)
    # the third item reaches below the first two round-offs by more than a
    # significand, so adding the round-offs rounds
    span = 4 * np.finfo(dtype).nmant
    worst = 0.0
    for _ in range(8000):
        x3 = rng.uniform(-1, 1) * 2.0 ** -int(rng.integers(1, span))
        xs = np.array([1.0, rng.uniform(0.5, 1.0), x3], dtype=dtype)
        v, e = oracle.seq("sumt", xs)
        A = float(np.sum(np.abs(xs.astype(np.float64))))
        r = float(_err(v, e, xs)) / bounds.tree_bound(dtype, 3, 0, A)
        assert r <= 1.0, r
        worst = max(worst, r)
    assert worst > 1.0 / 40, worst


@pytest.mark.parametrize("dtype", DTYPES)
def test_rigorous_tree_bound_is_approached(dtype):
    """The GPU order (order model) on a few hundred items of wide dynamic
    range, one and two blocks of one wave: every rigorous result within the
    bound of its tree, the largest at least 1/500 of it."""
    rng = np.random.default_rng(2)
    worst = 0.0
    for _ in range(600):
        n = int(rng.integers(8, 600))
        x = (rng.uniform(-1, 1, n) * 2.0 ** rng.integers(-30, 30, n)).astype(dtype)
        gb = int(rng.integers(1, 3))
        v, e = oracle.model_single("rigorous", x, None, 0, 64, 1, gb)
        ex = oracle.Exact(x)
        r = abs(ex.diff(v, e)) / bounds.single_bound(dtype, n, 64, 1, gb, ex.A)
        assert r <= 1.0, r
        worst = max(worst, r)
    assert worst > 1.0 / 500, worst


def test_double_word_bound_is_approached():
    """One double-word addition (DWPlusFP, AccurateDWPlusDW) against the
    double-word bound of a one-addition chain (3u^2 relative): the largest
    errors reach a fifth of it, none exceeds it."""
    rng = np.random.default_rng(4)
    worst_fp = worst_dw = 0.0
    for _ in range(6000):
        h = 1.0
        l = rng.uniform(-1, 1) * 2.0 ** -53
        x = rng.uniform(-1, 1) * 2.0 ** -int(rng.integers(1, 60))
        hh, ll = oracle.dw_plus_fp(h, l, x)
        r = float(_err(hh, ll, (h, l, x))) / bounds.dw_bound(1, 0, abs(h) + abs(l) + abs(x))
        assert r <= 1.0, r
        worst_fp = max(worst_fp, r)
        yh = rng.uniform(-1, 1) * 2.0 ** -int(rng.integers(0, 30))
        yl = rng.uniform(-1, 1) * abs(yh) * 2.0 ** -53
        hh, ll = oracle.dw_plus_dw(h, l, yh, yl)
        A = abs(h) + abs(l) + abs(yh) + abs(yl)
        r = float(_err(hh, ll, (h, l, yh, yl))) / bounds.dw_bound(1, 0, A)
        assert r <= 1.0, r
        worst_dw = max(worst_dw, r)
    assert worst_fp > 0.2 and worst_dw > 0.05, (worst_fp, worst_dw)
