"""The precision monitor's oracle (oracle/monitor.py), pinned by the paper's
own example, and the library's host-side argument checks (no GPU)."""
import ctypes
import json
import os

import numpy as np

import oracle
import synth
from oracle import monitor
from paper_1401_0248_amd import _lib
from paper_1401_0248_amd._lib import EALIGN, EINVAL

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hundred_hours.json")


def test_hundred_hours_is_flagged_in_binary32_only():
    """The paper's "100 hours" counter: binary32 twofold ends with an error
    term of 3.54 h on a value of 96.4 h (its table), the case the paper
    would interrupt and move to double. The same ticks summed in binary64
    leave an error term far below any sensible threshold."""
    g = json.load(open(GOLDEN))["rows"]["Twofold"]
    x = synth.hundred_hours()
    v, e = oracle.seq("sumtf", x)
    assert float("%.6g" % (float(e) / 3600)) == float(g["estimate"])
    assert monitor.flag(v, e, x.size, 1e-3, np.float32) == monitor.FLAG_ERROR
    v64, e64 = oracle.seq("sumtf", x.astype(np.float64))
    assert abs(float(e64)) < 1e-6 * abs(float(v64))
    assert monitor.flag(v64, e64, x.size, 1e-3, np.float64) == 0
    # the relative error term (3.7%) lies between two thresholds
    rel = abs(float(e)) / abs(float(v))
    assert monitor.flag(v, e, x.size, rel * 1.001, np.float32) == 0
    assert monitor.flag(v, e, x.size, rel * 0.999, np.float32) == monitor.FLAG_ERROR


def test_threshold_is_strict():
    v = 3.0
    for tau in (0.0, 0.25, 1e-7):
        e = tau * abs(v)
        assert monitor.flag(v, e, 1, tau, np.float64) == 0
        assert monitor.flag(v, np.nextafter(e, np.inf) if e else 5e-324, 1, tau,
                            np.float64) == monitor.FLAG_ERROR
    assert monitor.flag(0.0, 0.0, 1, 0.0, np.float64) == 0
    assert monitor.flag(0.0, -1e-300, 1, 1e300, np.float64) == monitor.FLAG_ERROR


def test_length_flag_at_one_over_u():
    assert monitor.flag(1.0, 0.0, 2 ** 24 - 1, 1.0, np.float32) == 0
    assert monitor.flag(1.0, 0.0, 2 ** 24, 1.0, np.float32) == monitor.FLAG_LENGTH
    assert monitor.flag(1.0, 0.0, 2 ** 24, 1.0, np.float64) == 0
    assert monitor.flag(1.0, 0.0, 2 ** 53, 1.0, np.float64) == monitor.FLAG_LENGTH


def test_nonfinite():
    for v, e in ((np.inf, 0.0), (1.0, np.nan), (-np.inf, np.inf), (np.nan, np.nan)):
        assert monitor.flag(v, e, 1, 0.5, np.float64) == monitor.FLAG_NONFINITE
    assert monitor.flag(np.inf, 0.0, 2 ** 24, 0.5, np.float32) == \
        monitor.FLAG_NONFINITE | monitor.FLAG_LENGTH


def test_monitor_argument_checks():
    L = _lib.load()
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: checks fail first
    odd = ctypes.c_void_p(0x10002)
    cnt = ctypes.c_void_p(0x20000)
    assert L.twofold_monitor(2, fake, 4, None, 8, 0.5, fake, cnt, None) == EINVAL  # dtype
    assert L.twofold_monitor(4, fake, -1, None, 8, 0.5, fake, cnt, None) == EINVAL
    assert L.twofold_monitor(4, None, 4, None, 8, 0.5, fake, cnt, None) == EINVAL
    assert L.twofold_monitor(4, fake, 4, None, 8, 0.5, None, cnt, None) == EINVAL
    assert L.twofold_monitor(4, fake, 4, None, 8, 0.5, fake, None, None) == EINVAL
    assert L.twofold_monitor(4, fake, 4, None, -1, 0.5, fake, cnt, None) == EINVAL
    for tau in (-1.0, float("nan"), float("inf")):
        assert L.twofold_monitor(4, fake, 4, None, 8, tau, fake, cnt, None) == EINVAL
    assert L.twofold_monitor(8, ctypes.c_void_p(0x10004), 4, None, 8, 0.5, fake, cnt, None) == EALIGN
    assert L.twofold_monitor(4, fake, 4, odd, 8, 0.5, fake, cnt, None) == EALIGN
    assert L.twofold_monitor(4, fake, 4, None, 8, 0.5, odd, cnt, None) == EALIGN
