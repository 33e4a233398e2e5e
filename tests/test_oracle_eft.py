"""Pins of the oracle's per-element steps against exact rational arithmetic.

Theorem 2 (Knuth's two-sum, section "Algorithms"): the rigorous step
captures the round-off of s + item exactly, for any operands. Theorem 1
(Dekker): the fast step is exact when |s| >= |item|, and may lose part of
the round-off otherwise. The dot step's remainder fma(x, y, -fl(x*y)) makes
fl(x*y) + remainder equal to x*y exactly. Each check runs the oracle's C
loops on two- or one-element inputs and compares with fractions.Fraction,
an implementation independent of the oracle.
"""
import math
import random
from fractions import Fraction

import numpy as np
import pytest

import oracle

F = Fraction


def _edge_values(dtype):
    fi = np.finfo(dtype)
    one = dtype(1)
    eps = fi.eps  # 2u
    vals = [dtype(0), one, -one, one + eps, one - eps / 2, dtype(3), dtype(0.1), dtype(-0.7),
            fi.tiny, fi.tiny * 3, fi.smallest_subnormal, fi.smallest_subnormal * 5,
            dtype(2) ** (fi.nmant), dtype(2) ** (fi.nmant + 1), dtype(2) ** (-fi.nmant),
            fi.max / 4, dtype(1.5) * eps, dtype(0.25) + eps / 8]
    out = []
    for v in vals:
        out += [dtype(v), dtype(-v)]
    return out


def _random_values(dtype, rng, count):
    p = np.finfo(dtype).nmant + 1
    out = []
    for _ in range(count):
        m = rng.integers(-(2 ** p) + 1, 2 ** p)
        e = int(rng.integers(-40, 40))
        out.append(dtype(math.ldexp(float(m), e - p)))
    return out


def _pairs(dtype):
    rng = np.random.default_rng(123)
    vals = _edge_values(dtype)
    pairs = [(a, b) for a in vals for b in vals]
    r = _random_values(dtype, rng, 600)
    pairs += list(zip(r[::2], r[1::2]))
    # exponent gaps 0, 1, p-1, p, p+1 around 1
    p = np.finfo(dtype).nmant + 1
    for gap in (0, 1, p - 1, p, p + 1, 2 * p):
        for _ in range(20):
            a = dtype(math.ldexp(float(rng.integers(2 ** (p - 1), 2 ** p)), -p + 1))
            b = dtype(math.ldexp(float(rng.integers(2 ** (p - 1), 2 ** p)), -p + 1 - gap))
            pairs += [(a, b), (b, a), (a, -b), (-b, a)]
    # keep finite sums only
    return [(a, b) for a, b in pairs if np.isfinite(np.array([a + b], dtype=dtype)).all()]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_rigorous_step_is_exact(dtype):
    """Theorem 2: value + error == a + b exactly, for every pair."""
    for a, b in _pairs(dtype):
        x = np.array([a, b], dtype=dtype)
        v, e = oracle.seq("sumt", x)
        assert F(float(v)) + F(float(e)) == F(float(a)) + F(float(b)), (a, b, v, e)
        # the value is the plain sum
        assert v == np.array([a], dtype=dtype)[0] + np.array([b], dtype=dtype)[0]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_fast_step_exact_when_ordered(dtype):
    """Theorem 1: exact whenever |a| >= |b| (the first item a becomes s)."""
    for a, b in _pairs(dtype):
        if abs(float(a)) < abs(float(b)):
            continue
        v, e = oracle.seq("sumtf", np.array([a, b], dtype=dtype))
        assert F(float(v)) + F(float(e)) == F(float(a)) + F(float(b)), (a, b)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_fast_step_loss_is_bounded(dtype):
    """When |a| < |b| the fast step may lose part of the round-off, but at
    most u(1+2u)|b| (u the unit roundoff)."""
    u = F(1, 2 ** (np.finfo(dtype).nmant + 1))
    for a, b in _pairs(dtype):
        v, e = oracle.seq("sumtf", np.array([a, b], dtype=dtype))
        loss = abs(F(float(v)) + F(float(e)) - F(float(a)) - F(float(b)))
        assert loss <= u * (1 + 2 * u) * abs(F(float(b))), (a, b, loss)


def test_fast_step_counterexample():
    """An unordered pair where the fast step is not exact but the rigorous
    one is: a = 0.25 + 2^-54, b = 1 - 2^-53."""
    a = 0.25 + 2.0 ** -54
    b = 1.0 - 2.0 ** -53
    x = np.array([a, b])
    v, e = oracle.seq("sumtf", x)
    assert v == 1.25 and e == -(2.0 ** -53)
    assert F(v) + F(e) != F(a) + F(b)
    v, e = oracle.seq("sumt", x)
    assert F(v) + F(e) == F(a) + F(b)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_dot_remainder_is_exact(dtype):
    """One-element dot: (value, error) = (fl(x*y), x*y - fl(x*y)) exactly, in
    both forms, as long as the product does not underflow."""
    rng = np.random.default_rng(7)
    vals = _random_values(dtype, rng, 400) + [dtype(0.1), dtype(3), dtype(-1) / dtype(3)]
    fi = np.finfo(dtype)
    for i in range(0, len(vals) - 1):
        a, b = vals[i], vals[i + 1]
        prod = F(float(a)) * F(float(b))
        if prod != 0 and abs(prod) < F(float(fi.tiny)) * 2 ** (fi.nmant + 1):
            continue
        for kind in ("dott", "dottf"):
            v, e = oracle.seq(kind, np.array([a], dtype=dtype), np.array([b], dtype=dtype))
            assert F(float(v)) + F(float(e)) == prod, (kind, a, b)
            assert v == (np.array([a], dtype=dtype) * np.array([b], dtype=dtype))[0]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_rigorous_dot_two_terms_exact(dtype):
    """Two-element rigorous dot: the products' remainders pi_i (|pi_i| <=
    u|p_i|) and the two-sum remainder d of p_1 + p_2 (|d| <= u|v|) are exact;
    only the two additions into e round. Hence
    |v + e - S| <= 3 u^2 (|v| + |p_1| + |p_2|)."""
    rng = np.random.default_rng(11)
    vals = _random_values(dtype, rng, 800)
    u = F(1, 2 ** (np.finfo(dtype).nmant + 1))
    for i in range(0, 796, 4):
        x = np.array(vals[i:i + 2], dtype=dtype)
        y = np.array(vals[i + 2:i + 4], dtype=dtype)
        S = sum(F(float(a)) * F(float(b)) for a, b in zip(x, y))
        p = x * y
        v, e = oracle.seq("dott", x, y)
        err = abs(F(float(v)) + F(float(e)) - S)
        bound = 3 * u * u * (abs(F(float(v))) + abs(F(float(p[0]))) + abs(F(float(p[1]))))
        assert err <= bound, (x, y, err, bound)
        # a dropped remainder would leave an error of order u|p|
        assert v == p[0] + p[1]


def test_kahan_matches_definition_small():
    """Kahan on [1, 2^-53, 2^-53] keeps the two small terms (Example 2):
    plain summation loses both."""
    x = np.array([1.0, 2.0 ** -53, 2.0 ** -53])
    assert oracle.seq("sum", x)[0] == 1.0
    assert oracle.seq("sumk", x)[0] == 1.0 + 2.0 ** -52


def test_random_pairs_python_floats():
    """Two-sum identity on random binary64 pairs with wide exponent ranges,
    drawn with Python's own generator."""
    rnd = random.Random(5)
    for _ in range(2000):
        a = rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-60, 60)
        b = rnd.uniform(-1, 1) * 2.0 ** rnd.randint(-60, 60)
        v, e = oracle.seq("sumt", np.array([a, b]))
        assert F(v) + F(e) == F(a) + F(b)


# ---- double-word additions (the wide accumulator for binary64 data) ----------
def _dw(rng, scale):
    """A random normalized double-word number (h, l), h = fl(h + l)."""
    h = float(rng.standard_normal() * 2.0 ** scale)
    l = float(rng.standard_normal()) * abs(h) * 2.0 ** -int(rng.integers(53, 60))
    hh, ll = oracle.dw_plus_fp(h, 0.0, l)  # renormalize
    return hh, ll


def test_dw_additions_within_published_bounds():
    """DWPlusFP within 2u^2 and AccurateDWPlusDW within 3u^2 + 13u^3 of the
    exact sum (Joldes, Muller, Popescu 2017, Algorithms 4 and 6), results
    normalized, on random pairs with cancellations and wide exponent gaps."""
    u = 2.0 ** -53
    rng = np.random.default_rng(31)
    for _ in range(4000):
        xh, xl = _dw(rng, int(rng.integers(-30, 30)))
        yh, yl = _dw(rng, int(rng.integers(-30, 30)))
        if rng.random() < 0.3:  # heavy cancellation
            yh, yl = oracle.dw_plus_fp(-xh, 0.0, xh * 2.0 ** -int(rng.integers(20, 60)))
        exact = F(xh) + F(xl) + F(yh) + F(yl)
        zh, zl = oracle.dw_plus_dw(xh, xl, yh, yl)
        assert zh == zh + zl
        assert abs(F(zh) + F(zl) - exact) <= (F(3 * u * u) + F(13) * F(u) ** 3) * abs(exact)
        y = float(yh)
        exact = F(xh) + F(xl) + F(y)
        zh, zl = oracle.dw_plus_fp(xh, xl, y)
        assert zh == zh + zl
        assert abs(F(zh) + F(zl) - exact) <= 2 * F(u) * F(u) * abs(exact)


def test_dw_step_catches_a_dropped_term():
    """The pins are sharp enough to see a mistake: dropping the low parts'
    two-sum remainder (tl) breaks the bound on some input."""
    u = 2.0 ** -53
    rng = np.random.default_rng(32)
    bad = 0
    for _ in range(2000):
        xh, xl = _dw(rng, 0)
        yh, yl = _dw(rng, 0)
        exact = F(xh) + F(xl) + F(yh) + F(yl)
        sh = xh + yh
        bv = sh - xh
        sl = (xh - (sh - bv)) + (yh - bv)
        th = xl + yl  # the two-sum remainder of the low parts is dropped
        c = sl + th
        vh = sh + c
        vl = c - (vh - sh)
        zh = vh + vl
        zl = vl - (zh - vh)
        if abs(F(zh) + F(zl) - exact) > (F(3 * u * u) + F(13) * F(u) ** 3) * abs(exact):
            bad += 1
    assert bad > 0
