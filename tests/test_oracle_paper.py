"""Pins of the oracle's sequential loops against what the paper prints and
what the mathematics fixes.

* The "100 hours" table (section "Accuracy"): every printed number.
* The twofold value is the direct sum in the same order (section
  "Algorithms", the text after Example 2): checked against numpy's
  sequential cumulative sum.
* On the binary64 grid 2^-52 (binary32: 2^-23) with |x| < 1, every
  round-off of a partial sum is a representable multiple of the grid, so
  value + error equals the exact sum in both forms ("exact-grid" sums).
* Rigorous dots satisfy |v + e - S| <= 4 N u^2 sum|x y|; the fast form stays
  within 4 N u^2 sum|xy| + 2u sum|xy| (Theorem 1's precondition may fail).
* Table 2a's qualitative picture: twofold is far more accurate than direct
  summation on 2^20 uniform values.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hundred_hours.json")


def _u(dtype):
    return 2.0 ** -(np.finfo(dtype).nmant + 1)


def test_hundred_hours_golden():
    g = json.load(open(GOLDEN))["rows"]
    x = synth.hundred_hours()
    hours = lambda sec: float(sec) / 3600.0  # noqa: E731

    v, _ = oracle.seq("sum", x)
    assert "%g" % hours(v) == g["Direct"]["result"]
    assert "%g" % (100.0 - hours(v)) == g["Direct"]["deviation"]

    d, _ = oracle.seq("sumd", x)
    assert "%g" % hours(d) == g["Double"]["result"]
    assert "%g" % abs(hours(d) - 100.0) == g["Double"]["deviation"]

    k, _ = oracle.seq("sumk", x)
    assert "%g" % hours(k) == g["Kahan"]["result"]
    assert "%g" % abs(hours(k) - 100.0) == g["Kahan"]["deviation"]

    for kind in ("sumtf", "sumt"):  # s >= y at every step: both forms agree
        v, e = oracle.seq(kind, x)
        r = float(v) + float(e)
        assert "%g" % hours(r) == g["Twofold"]["result"]
        assert "%g" % abs(hours(r) - 100.0) == g["Twofold"]["deviation"]
        assert "%g" % hours(e) == g["Twofold"]["estimate"]
        assert "%g" % hours(v) == g["Direct"]["result"]


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("kind", ["sumtf", "sumt"])
def test_value_is_direct_sum(dtype, kind):
    rng = np.random.default_rng(4)
    x = (rng.standard_normal(20000) * np.exp2(rng.integers(-20, 20, 20000))).astype(dtype)
    v, _ = oracle.seq(kind, x)
    assert v == np.cumsum(x, dtype=dtype)[-1]
    assert oracle.seq("sum", x)[0] == v


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("kind", ["dottf", "dott", "dottf_rounded", "dott_rounded"])
def test_dot_value_is_direct_dot(dtype, kind):
    rng = np.random.default_rng(5)
    x = rng.standard_normal(5000).astype(dtype)
    y = rng.standard_normal(5000).astype(dtype)
    v, _ = oracle.seq(kind, x, y)
    assert v == np.cumsum(x * y, dtype=dtype)[-1]
    assert oracle.seq("dot", x, y)[0] == v


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("kind", ["sumtf", "sumt"])
def test_exact_grid_sums(dtype, kind):
    x = synth.uniform(0, 1 << 16, dtype)
    ex = oracle.Exact(x)
    v, e = oracle.seq(kind, x)
    assert ex.diff(float(v), float(e)) == 0.0
    assert ex.diff(float(v)) != 0.0  # the value alone is not exact


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_rigorous_dot_bound(dtype):
    u = _u(dtype)
    for seed in range(3):
        x, y = synth.uniform(seed, 1 << 14, dtype, count=2)
        ex = oracle.Exact(x, y)
        v, e = oracle.seq("dott", x, y)
        D = abs(ex.diff(float(v), float(e)))
        assert D <= 4 * x.size * u * u * ex.A
        # the error explains most of the value's deviation
        assert abs(ex.diff(float(v))) > 10 * D


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_fast_dot_apriori_bound(dtype):
    u = _u(dtype)
    x, y = synth.uniform(9, 1 << 14, dtype, count=2)
    ex = oracle.Exact(x, y)
    v, e = oracle.seq("dottf", x, y)
    D = abs(ex.diff(float(v), float(e)))
    assert D <= 4 * x.size * u * u * ex.A + 2 * u * ex.A


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_rounded_product_dot_misses_product_error(dtype):
    """The paper's dot feeds the rounded product: its error does not see the
    products' round-offs, so it misses by far more than the FMA form."""
    x, y = synth.uniform(12, 1 << 14, dtype, count=2)
    ex = oracle.Exact(x, y)
    v1, e1 = oracle.seq("dott_rounded", x, y)
    v2, e2 = oracle.seq("dott", x, y)
    assert v1 == v2
    assert abs(ex.diff(float(v1), float(e1))) > 100 * abs(ex.diff(float(v2), float(e2)))


def test_illconditioned_rigorous_bound():
    for dtype in (np.float32, np.float64):
        u = _u(dtype)
        for d in (6, 10, 16):
            x, y = synth.illcond_dot(synth.illcond_seed(d), 1 << 14, 10.0 ** d, dtype)
            ex = oracle.Exact(x, y)
            v, e = oracle.seq("dott", x, y)
            assert abs(ex.diff(float(v), float(e))) <= 4 * x.size * u * u * ex.A


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_table2a_magnitudes(dtype):
    """Twofold fast summation of 2^20 uniform [-1, 1) values is orders of
    magnitude more accurate than direct summation (table of section
    "Accuracy"; the paper's generators and seeds are not reproducible, so
    only the ordering is pinned)."""
    x = synth.uniform(0, 1 << 20, dtype)
    ex = oracle.Exact(x)
    v, e = oracle.seq("sumtf", x)
    direct = abs(ex.diff(float(oracle.seq("sum", x)[0])))
    twofold = abs(ex.diff(float(v) + float(e)))
    assert twofold * 1e3 < direct
    kahan = abs(ex.diff(float(oracle.seq("sumk", x)[0])))
    assert kahan < direct


def test_sumd_dotd_are_exact_products():
    x, y = synth.uniform(3, 4096, np.float32, count=2)
    s = oracle.seq("dotd", x, y)[0]
    assert s == np.cumsum(x.astype(np.float64) * y.astype(np.float64))[-1]
    assert oracle.seq("sumd", x)[0] == np.cumsum(x.astype(np.float64))[-1]
