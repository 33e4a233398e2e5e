"""Pins of the oracle's exact accumulator against independent references:
math.fsum (CPython's correctly rounded summation of binary64 values),
fractions.Fraction (exact rationals), integer closed forms and the paper's
"100 hours" exact total (section "Accuracy")."""
import math
from fractions import Fraction as F

import numpy as np
import pytest

import oracle


def _fraction_round(fr):
    """Nearest binary64 to a Fraction (Python rounds int/int divisions
    correctly)."""
    return fr.numerator / fr.denominator if fr.denominator != 1 else float(fr.numerator)


def test_sum_matches_fsum_random():
    rng = np.random.default_rng(1)
    for trial in range(20):
        n = int(rng.integers(1, 5000))
        e = rng.integers(-300, 300, size=n)
        x = rng.standard_normal(n) * np.exp2(e.astype(np.float64))
        ex = oracle.Exact(x, nthreads=1 + trial % 4)
        assert ex.S == math.fsum(x.tolist())
        assert ex.A == math.fsum(np.abs(x).tolist())


def test_sum_heavy_cancellation():
    x = np.array([1e300, 1.0, -1e300, 2.0 ** -1074, 3.0, -1.0])
    ex = oracle.Exact(x)
    assert ex.S == math.fsum(x.tolist()) == 3.0
    assert ex.diff(3.0) == -(2.0 ** -1074)
    assert ex.sign == 1


def test_sum_subnormals_and_ties():
    # ties to even: 1 + 2^-53 rounds to 1; anything above the tie rounds up
    assert oracle.Exact(np.array([1.0, 2.0 ** -53])).S == 1.0
    assert oracle.Exact(np.array([1.0, 2.0 ** -53, 2.0 ** -1000])).S == 1.0 + 2.0 ** -52
    assert oracle.Exact(np.array([1.0 + 2.0 ** -52, 2.0 ** -53])).S == 1.0 + 2.0 ** -51
    tiny = 2.0 ** -1074
    x = np.array([tiny] * 7 + [-2 * tiny])
    assert oracle.Exact(x).S == 5 * tiny
    x = np.array([2.0 ** -1022, -tiny])
    assert oracle.Exact(x).S == 2.0 ** -1022 - tiny
    assert oracle.Exact(np.zeros(10)).S == 0.0
    assert oracle.Exact(np.array([-0.0])).sign == 0


def test_sum_overflow_rounding():
    big = np.finfo(np.float64).max
    assert oracle.Exact(np.array([big, big, -big])).S == big
    assert math.isinf(oracle.Exact(np.array([big, big])).S)


def test_nonfinite():
    assert math.isnan(oracle.Exact(np.array([1.0, np.nan])).S)
    assert oracle.Exact(np.array([1.0, np.inf])).S == math.inf
    assert math.isnan(oracle.Exact(np.array([np.inf, -np.inf])).S)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_dot_matches_fraction(dtype):
    rng = np.random.default_rng(2)
    for trial in range(6):
        n = int(rng.integers(1, 1500))
        x = (rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, n).astype(float))).astype(dtype)
        y = (rng.standard_normal(n) * np.exp2(rng.integers(-60, 60, n).astype(float))).astype(dtype)
        exact = sum(F(float(a)) * F(float(b)) for a, b in zip(x, y))
        ex = oracle.Exact(x, y, nthreads=1 + trial % 3)
        assert ex.S == _fraction_round(exact)
        assert ex.A == _fraction_round(sum(abs(F(float(a)) * F(float(b))) for a, b in zip(x, y)))
        v = float(np.float64(rng.standard_normal()))
        assert ex.diff(v) == _fraction_round(F(v) - exact)


def test_dot_extreme_exponents():
    """Products of subnormals and of huge values stay exact."""
    tiny = 2.0 ** -1074
    x = np.array([tiny, 2.0 ** 1000, 3.0])
    y = np.array([tiny, 2.0 ** 1000, -1.0])
    ex = oracle.Exact(x, y)
    # exact value 2^2000 - 3 + 2^-2148 is above the binary64 range
    assert ex.S == math.inf and ex.sign == 1
    x = np.array([tiny, tiny])
    y = np.array([tiny, -tiny])
    assert oracle.Exact(x, y).S == 0.0
    x = np.array([2.0 ** -600, 1.0])
    y = np.array([2.0 ** -600, -1.0])
    ex = oracle.Exact(x, y)
    assert ex.S == -1.0
    assert ex.diff(-1.0) == -(2.0 ** -1200)


def test_integer_closed_form():
    n = 100000
    x = np.arange(1, n + 1, dtype=np.float64)
    assert oracle.Exact(x).S == n * (n + 1) // 2
    # sum of squares via the dot
    assert oracle.Exact(x, x).S == n * (n + 1) * (2 * n + 1) // 6
    # alternating sign, exact zero
    z = np.concatenate([x, -x])
    assert oracle.Exact(z).S == 0.0 and oracle.Exact(z).sign == 0


def test_hundred_hours_exact_total():
    """3.6e6 * fl32(0.1) = 377487365625 / 2^20 seconds exactly."""
    x = np.full(3_600_000, np.float32(0.1), dtype=np.float32)
    ex = oracle.Exact(x)
    assert F(ex.S) == F(377487365625, 2 ** 20)
    assert ex.S32 == np.float32(360000.0)


def test_f32_rounding():
    # halfway between binary32 neighbours of 1: 1 + 2^-24 rounds to 1
    x = np.array([1.0, 2.0 ** -24], dtype=np.float32)
    assert oracle.Exact(x).S32 == np.float32(1.0)
    x = np.array([1.0, 2.0 ** -24, 2.0 ** -60], dtype=np.float32)
    assert oracle.Exact(x).S32 == np.float32(1.0) + np.float32(2.0 ** -23)
    assert oracle.Exact(np.array([1e-45], dtype=np.float32)).S32 == np.float32(1e-45)


def test_thread_count_independent():
    rng = np.random.default_rng(3)
    x = rng.standard_normal(200001) * 1e10
    y = rng.standard_normal(200001)
    vals = {oracle.Exact(x, y, nthreads=t).diff(0.1) for t in (1, 2, 7, 16)}
    assert len(vals) == 1
