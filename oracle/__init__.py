"""CPU oracle for twofold summation and dot products.

TEST INFRASTRUCTURE: only the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package. The GPU library
neither imports nor links it, and the two share no code.

Three parts, all in plain C (``liboracle.so``, built by ``oracle/build.py``):

* ``Exact``: an exact fixed-point accumulator defining the target
  S = sum x_n or sum x_n*y_n and A = sum |x_n| or sum |x_n*y_n|
  (the exact real that the paper's value + error pair approximates,
  "Overview").
* ``seq``: the paper's sequential methods (section "Algorithms": Example 1
  ``sumtf``, Example 2 ``sumk``, Example 3 ``sumt`` and direct ``sum``, the
  double accumulator ``sumd``, and dot products summing the rounded
  products x_i*y_i as items), restated on fast-two-sum and two-sum
  (Theorems 1 and 2), plus the dot with an FMA remainder, and for
  binary64 data the double-word accumulator ``sumdd``/``dotdd`` standing in
  for the paper's quad one (``dw_plus_fp``/``dw_plus_dw`` expose its steps).
* ``model_single`` / ``model_seg``: the same per-element steps applied in the
  GPU library's documented reduction order, for bitwise comparisons.
"""
import ctypes
import os

import numpy as np

from . import build as _build

PLAIN, FAST, RIGOROUS, WIDE, KAHAN, FAST_ROUNDED, RIGOROUS_ROUNDED, MIXED = 0, 1, 2, 3, 4, 5, 6, 7
MODES = {"plain": PLAIN, "fast": FAST, "rigorous": RIGOROUS, "wide": WIDE, "kahan": KAHAN,
         "fast_rounded": FAST_ROUNDED, "rigorous_rounded": RIGOROUS_ROUNDED, "mixed": MIXED}

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.build()
        L = ctypes.CDLL(path)
        vp, i64, i32, dp = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.POINTER(ctypes.c_double)
        L.oracle_xacc_size.restype = ctypes.c_size_t
        L.oracle_xacc_size.argtypes = []
        L.oracle_xacc_clear.argtypes = [vp]
        for nm in ("oracle_xacc_add_sum_f32", "oracle_xacc_add_sum_f64"):
            getattr(L, nm).argtypes = [vp, vp, i64, i32, i32]
        for nm in ("oracle_xacc_add_dot_f32", "oracle_xacc_add_dot_f64"):
            getattr(L, nm).argtypes = [vp, vp, vp, i64, i32, i32]
        L.oracle_xacc_round.restype = ctypes.c_double
        L.oracle_xacc_round.argtypes = [vp, i32, i32]
        L.oracle_xacc_round_diff.restype = ctypes.c_double
        L.oracle_xacc_round_diff.argtypes = [vp, dp, i32]
        L.oracle_xacc_sign.restype = i32
        L.oracle_xacc_sign.argtypes = [vp]
        for sfx, ct in (("f32", ctypes.c_float), ("f64", ctypes.c_double)):
            for nm in ("sum", "sumk"):
                f = getattr(L, "oracle_%s_%s" % (nm, sfx))
                f.restype = ct
                f.argtypes = [vp, i64]
            for nm in ("sumtf", "sumt", "sumk_pair"):
                f = getattr(L, "oracle_%s_%s" % (nm, sfx))
                f.restype = None
                f.argtypes = [vp, i64, vp]
            for nm in ("dot", "dotk"):
                f = getattr(L, "oracle_%s_%s" % (nm, sfx))
                f.restype = ct
                f.argtypes = [vp, vp, i64]
            for nm in ("dottf_rounded", "dott_rounded", "dottf", "dott", "dotk_pair"):
                f = getattr(L, "oracle_%s_%s" % (nm, sfx))
                f.restype = None
                f.argtypes = [vp, vp, i64, vp]
        L.oracle_sumd_f32.restype = ctypes.c_double
        L.oracle_sumd_f32.argtypes = [vp, i64]
        L.oracle_dotd_f32.restype = ctypes.c_double
        L.oracle_dotd_f32.argtypes = [vp, vp, i64]
        L.oracle_sumdd_f64.restype = None
        L.oracle_sumdd_f64.argtypes = [vp, i64, vp]
        L.oracle_dotdd_f64.restype = None
        L.oracle_dotdd_f64.argtypes = [vp, vp, i64, vp]
        cd = ctypes.c_double
        L.oracle_dw_plus_fp.restype = None
        L.oracle_dw_plus_fp.argtypes = [cd, cd, cd, vp]
        L.oracle_dw_plus_dw.restype = None
        L.oracle_dw_plus_dw.argtypes = [cd, cd, cd, cd, vp]
        L.oracle_model_single.restype = i32
        L.oracle_model_single.argtypes = [i32, i32, vp, vp, i64, i32, i32, i32, i32, vp, vp]
        L.oracle_model_seg.restype = i32
        L.oracle_model_seg.argtypes = [i32, i32, vp, vp, vp, i64, i32, i32, i64, vp, vp]
        _lib = L
    return _lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


def _check(x, y=None):
    x = np.ascontiguousarray(x)
    if x.dtype not in (np.float32, np.float64):
        raise TypeError("oracle: dtype must be float32 or float64, got %s" % x.dtype)
    if y is not None:
        y = np.ascontiguousarray(y)
        if y.dtype != x.dtype or y.shape != x.shape:
            raise ValueError("oracle: x and y must share dtype and shape")
    return x, y


def default_threads():
    return max(1, min(16, os.cpu_count() or 1))


class Exact:
    """Exact S and A of a sum (y is None) or dot, by integer accumulation."""

    def __init__(self, x, y=None, nthreads=None):
        x, y = _check(x, y)
        L = lib()
        nt = default_threads() if nthreads is None else nthreads
        sz = L.oracle_xacc_size()
        self._S = ctypes.create_string_buffer(sz)
        self._A = ctypes.create_string_buffer(sz)
        self.n = x.size
        self.dtype = x.dtype
        sfx = "f32" if x.dtype == np.float32 else "f64"
        for buf, absval in ((self._S, 0), (self._A, 1)):
            L.oracle_xacc_clear(buf)
            if y is None:
                getattr(L, "oracle_xacc_add_sum_" + sfx)(buf, _ptr(x), x.size, absval, nt)
            else:
                getattr(L, "oracle_xacc_add_dot_" + sfx)(buf, _ptr(x), _ptr(y), x.size, absval, nt)

    @property
    def S(self):
        """S rounded to nearest binary64."""
        return lib().oracle_xacc_round(self._S, 53, -1074)

    @property
    def S32(self):
        """S rounded to nearest binary32 (returned as a float32)."""
        return np.float32(lib().oracle_xacc_round(self._S, 24, -149))

    @property
    def A(self):
        """A = sum of absolute terms, rounded to nearest binary64."""
        return lib().oracle_xacc_round(self._A, 53, -1074)

    @property
    def sign(self):
        return lib().oracle_xacc_sign(self._S)

    def diff(self, *terms):
        """fl64(sum(terms) - S), computed exactly and rounded once."""
        arr = (ctypes.c_double * max(1, len(terms)))(*[float(t) for t in terms])
        return lib().oracle_xacc_round_diff(self._S, arr, len(terms))


def seq(kind, x, y=None):
    """Sequential paper loop ``kind`` on x (and y). Returns (value, error)
    as numpy scalars of the data type (error 0 for single-result loops);
    ``sumd``/``dotd`` return binary64 values."""
    x, y = _check(x, y)
    L = lib()
    sfx = "f32" if x.dtype == np.float32 else "f64"
    f = getattr(L, "oracle_%s_%s" % (kind, sfx))
    if kind in ("sum", "sumk", "sumd"):
        v = f(_ptr(x), x.size)
        t = np.float64 if kind == "sumd" else x.dtype.type
        return t(v), t(0)
    if kind in ("dot", "dotk", "dotd"):
        v = f(_ptr(x), _ptr(y), x.size)
        t = np.float64 if kind == "dotd" else x.dtype.type
        return t(v), t(0)
    out = np.zeros(2, dtype=x.dtype)
    if kind in ("sumtf", "sumt", "sumk_pair", "sumdd"):
        f(_ptr(x), x.size, _ptr(out))
    else:
        f(_ptr(x), _ptr(y), x.size, _ptr(out))
    return out[0], out[1]


def dw_plus_fp(h, l, y):
    """DWPlusFP (Joldes, Muller, Popescu 2017, Algorithm 4): (h, l) + y."""
    out = np.zeros(2)
    lib().oracle_dw_plus_fp(h, l, y, _ptr(out))
    return float(out[0]), float(out[1])


def dw_plus_dw(xh, xl, yh, yl):
    """AccurateDWPlusDW (same paper, Algorithm 6): (xh, xl) + (yh, yl)."""
    out = np.zeros(2)
    lib().oracle_dw_plus_dw(xh, xl, yh, yl, _ptr(out))
    return float(out[0]), float(out[1])


def model_single(mode, x, y=None, x_misalign=0, block_threads=256, unroll=4, grid_blocks=1,
                 with_violations=False):
    """(value, error) of the single-vector reduction in the GPU order. With
    with_violations, also the fast forms' sum of |item| over the steps that
    break Theorem 1's condition (see ``fast_loss_bound``)."""
    x, y = _check(x, y)
    out = np.zeros(2, dtype=np.float64)
    viol = np.zeros(1, dtype=np.float64)
    rc = lib().oracle_model_single(x.itemsize, MODES.get(mode, mode), _ptr(x), _ptr(y), x.size,
                                   x_misalign, block_threads, unroll, grid_blocks, _ptr(out),
                                   _ptr(viol))
    if rc != 0:
        raise ValueError("oracle_model_single rejected its arguments")
    return (out, float(viol[0])) if with_violations else out


def model_seg(mode, x, offsets, y=None, x_misalign=0, unroll=4, tile_elems=4096,
              with_violations=False):
    """(nseg, 2) array of (value, error) of the segmented reduction in the
    GPU order (and, with with_violations, the per-segment violation sums)."""
    x, y = _check(x, y)
    off = np.ascontiguousarray(offsets, dtype=np.int64)
    nseg = off.size - 1
    out = np.zeros((max(nseg, 0), 2), dtype=np.float64)
    viol = np.zeros(max(nseg, 1), dtype=np.float64)
    rc = lib().oracle_model_seg(x.itemsize, MODES.get(mode, mode), _ptr(x), _ptr(y), _ptr(off), nseg,
                                x_misalign, unroll, tile_elems, _ptr(out), _ptr(viol))
    if rc != 0:
        raise ValueError("oracle_model_seg rejected its arguments")
    return (out, viol[:max(nseg, 0)].copy()) if with_violations else out
