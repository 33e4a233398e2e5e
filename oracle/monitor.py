"""Precision monitor, written from the paper (test infrastructure, like the
rest of this package).

The paper proposes to interrupt a computation when its error term gets too
large, as a sign that the precision in use is not enough and that a wider
type (double instead of float) may be needed ("Algorithms", remarks after
the rigorous form). It also expects twofold summation to work for N below
1/u: 2^24 in binary32, 2^53 in binary64 ("Overview"). For one result
(value v, error e, length N) and a threshold tau >= 0:

* ERROR     when v and e are finite and |e| > tau * |v|;
* LENGTH    when N >= 1/u;
* NONFINITE when v or e is Inf or NaN.

v and e are taken as binary64 numbers (binary32 pairs widen exactly), and
tau * |v| is one binary64 multiplication, as Python floats compute it.
"""
import math

import numpy as np

FLAG_ERROR, FLAG_LENGTH, FLAG_NONFINITE = 1, 2, 4


def inv_unit_roundoff(dtype):
    return 2 ** (np.finfo(dtype).nmant + 1)


def flag(v, e, length, tau, dtype):
    v, e = float(v), float(e)
    f = 0
    if not (math.isfinite(v) and math.isfinite(e)):
        f |= FLAG_NONFINITE
    elif abs(e) > tau * abs(v):
        f |= FLAG_ERROR
    if length >= inv_unit_roundoff(dtype):
        f |= FLAG_LENGTH
    return f


def flags(pairs, lengths, tau, dtype):
    """Flags of every (value, error) row of pairs with the given lengths."""
    return [flag(p[0], p[1], int(n), tau, dtype) for p, n in zip(pairs, lengths)]
