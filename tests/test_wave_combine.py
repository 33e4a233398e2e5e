"""The wave combine's two schedules give the same pair (CPU).

The documented order (include/twofold.h, step 5) lets every lane l replace
its pair by combine(P_l, P_{l xor d}) for d = 1, 2, 4, ..., 32 and reads
lane 0. The kernels move pairs with DPP row_shr:d (d <= 8, within rows of
16 lanes), row_bcast:15 and row_bcast:31 instead: the top lane of each
aligned group of 2d lanes combines the received pair (from lane l - d, or
lane 15 of the row before, or lane 31) with its own, the received one
first, and lane 63 holds the result. Both are the balanced tree over the 64
lanes with the lower half first in every combine; this test checks that
claim bit for bit on random pairs, with the combines the modes use, written
out here from Theorem 2 (two-sum) in numpy scalars. The GPU tests check
the kernels' pairs against the order model, which follows the xor form.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def two_sum(a, b):
    s = a + b
    bv = s - a
    av = s - bv
    return s, (a - av) + (b - bv)


def combine_rigorous(p, q):
    s, d = two_sum(p[0], q[0])
    return s, (p[1] + q[1]) + d


def combine_plain(p, q):
    return p[0] + q[0], type(p[0])(0)


def xor_exchange(pairs, combine):
    P = list(pairs)
    for d in (1, 2, 4, 8, 16, 32):
        P = [combine(P[l], P[l ^ d]) for l in range(64)]
    return P[0]


def dpp_exchange(pairs, combine):
    P = list(pairs)
    for d in (1, 2, 4, 8):  # row_shr:d, rows of 16 lanes
        Q = list(P)
        for l in range(64):
            if l % 16 >= d:
                Q[l] = combine(P[l - d], P[l])
        P = Q
    Q = list(P)  # row_bcast:15 into rows 1 and 3
    for l in list(range(16, 32)) + list(range(48, 64)):
        Q[l] = combine(P[(l // 16) * 16 - 1], P[l])
    P = Q
    Q = list(P)  # row_bcast:31 into rows 2 and 3
    for l in range(32, 64):
        Q[l] = combine(P[31], P[l])
    return Q[63]


def bits(p):
    return tuple(np.asarray(v).tobytes() for v in p)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("combine", [combine_rigorous, combine_plain])
def test_dpp_schedule_equals_xor_schedule(dtype, combine):
    rng = np.random.default_rng(5)
    for trial in range(200):
        # values over many binades, signs mixed, some exact cancellations and
        # zeros, small error terms
        v = (rng.uniform(-1, 1, 64) * 2.0 ** rng.integers(-30, 30, 64)).astype(dtype)
        if trial % 5 == 0:
            v[rng.integers(0, 64, 8)] = 0
        if trial % 7 == 0:
            v[32:] = -v[:32]
        e = (v * rng.uniform(-1, 1, 64) * 2.0 ** -30).astype(dtype)
        pairs = [(v[l], e[l]) for l in range(64)]
        assert bits(xor_exchange(pairs, combine)) == bits(dpp_exchange(pairs, combine)), trial


def chain(pairs, combine):
    acc = pairs[0]
    for p in pairs[1:]:
        acc = combine(acc, p)
    return acc


def test_check_tells_trees_apart():
    # the comparison has teeth: another tree over the same pairs (a
    # left-to-right chain) differs on some inputs. (The operand order inside
    # one combine does not matter: two-sum's remainder is exact either way.)
    rng = np.random.default_rng(6)
    diff = 0
    for trial in range(100):
        v = (rng.uniform(-1, 1, 64) * 2.0 ** rng.integers(-30, 30, 64)).astype(np.float32)
        e = (v * np.float32(2.0 ** -30)).astype(np.float32)
        pairs = [(v[l], e[l]) for l in range(64)]
        diff += bits(xor_exchange(pairs, combine_rigorous)) != bits(chain(pairs, combine_rigorous))
    assert diff > 0
