"""Seeded synthetic inputs for the twofold library's tests and benchmark.

Shared by the oracle side and the GPU side; holds none of the summation
arithmetic. Every draw comes from numpy's PCG64 raw 64-bit stream
(``Generator.bit_generator.random_raw``), which numpy keeps stable across
versions, followed by a fixed integer transform, so the same seed gives the
same bits everywhere:

* uniform(-1, 1) on the data type's grid:
  binary64 ``x = (raw >> 11) * 2**-52 - 1``, binary32
  ``x = (raw >> 40) * 2**-23 - 1``; both exact, in [-1, 1);
* uniform integer in [lo, hi]: ``lo + (((raw >> 32) * (hi - lo + 1)) >> 32)``;
* uniform real in [0, 1): ``(raw >> 11) * 2**-53``.

Arrays are drawn whole and in a fixed order (x before y, mantissas before
exponents) so each recipe is a pure function of its seed.
"""
import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libsynth.so")
_lib = None


def build(force=False):
    src = os.path.join(HERE, "illcond.c")
    if not force and os.path.exists(_LIB_PATH) and os.path.getmtime(_LIB_PATH) >= os.path.getmtime(src):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-o", tmp, src, "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("synth build failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _clib():
    global _lib
    if _lib is None:
        # TWOFOLD_SYNTH_LIB: another build of illcond.c (the sanitizer test's)
        L = ctypes.CDLL(os.environ.get("TWOFOLD_SYNTH_LIB") or build())
        vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        for nm in ("synth_illcond_tail_f64", "synth_illcond_tail_f32"):
            f = getattr(L, nm)
            f.restype = i64
            f.argtypes = [vp, vp, i64, i64, vp, vp, i32, ctypes.c_double,
                          ctypes.POINTER(ctypes.c_double)]
        _lib = L
    return _lib


def _rng(seed):
    if isinstance(seed, (list, tuple)):
        seed = np.random.SeedSequence(list(seed))
    return np.random.Generator(np.random.PCG64(seed))


def raw(rng, n):
    return rng.bit_generator.random_raw(int(n))


def raw_to_uniform(r, dtype):
    """uniform(-1, 1) values on the grid of dtype, exact."""
    if np.dtype(dtype) == np.float64:
        return (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0
    k = (r >> np.uint64(40)).astype(np.float32)  # < 2^24: exact in binary32
    return (k * np.float32(2.0 ** -23) - np.float32(1.0)).astype(np.float32)


def raw_to_int(r, lo, hi):
    span = np.uint64(hi - lo + 1)
    return (((r >> np.uint64(32)) * span) >> np.uint64(32)).astype(np.int64) + lo


def raw_to_unit(r):
    return (r >> np.uint64(11)).astype(np.float64) * 2.0 ** -53


def uniform(seed, n, dtype, count=1):
    """``count`` arrays of n uniform(-1, 1) values (x first, then y)."""
    rng = _rng(seed)
    out = [raw_to_uniform(raw(rng, n), dtype) for _ in range(count)]
    return out[0] if count == 1 else out


def uniform_chunks(seed, n, dtype, chunk=1 << 24):
    """The same stream as ``uniform(seed, n, dtype)`` in pieces of at most
    ``chunk`` values, for inputs too large to materialise twice on the host."""
    rng = _rng(seed)
    done = 0
    while done < n:
        m = min(chunk, n - done)
        yield raw_to_uniform(raw(rng, m), dtype)
        done += m


def uniform_fill(seed, n, dtype, nthreads=None, out=None):
    """The same n values as ``uniform(seed, n, dtype)`` (one array: x and y
    of a dot drawn as one stream of 2n values), drawn by several threads.
    Thread t draws positions [a_t, b_t) of the stream from its own copy of
    the generator, advanced by a_t draws (PCG64's jump-ahead: one 64-bit
    draw per value), so the result does not depend on the thread count."""
    from concurrent.futures import ThreadPoolExecutor

    n = int(n)
    dtype = np.dtype(dtype)
    if out is None:
        out = np.empty(n, dtype=dtype)
    if nthreads is None:
        nthreads = max(1, min(16, os.cpu_count() or 1))
    chunk = 1 << 22
    starts = list(range(0, n, chunk))

    def part(a):
        m = min(chunk, n - a)
        bg = np.random.PCG64(seed)
        bg.advance(a)
        out[a:a + m] = raw_to_uniform(bg.random_raw(m), dtype)

    with ThreadPoolExecutor(max_workers=nthreads) as ex:
        list(ex.map(part, starts))
    return out


def scaled(seed, n, lo=-20, hi=20):
    """binary32 x, y with x = m * 2^k: m uniform(-1, 1), k uniform integer in
    [lo, hi]; draw order m_x, k_x, m_y, k_y. Every value is a multiple of
    2^(lo - 23), so x*y and its FMA remainder stay far from underflow."""
    rng = _rng(seed)
    out = []
    for _ in range(2):
        m = raw_to_uniform(raw(rng, n), np.float32)
        k = raw_to_int(raw(rng, n), lo, hi)
        out.append(np.ldexp(m, k.astype(np.int32)).astype(np.float32))
    return out[0], out[1]


def _illcond_once(mx, my, kx, ky, n, h, dtype, n_end=None):
    """The recipe on [0, n_end) (default n): first half random exponents,
    then the cancelling tail up to n_end. Elements from n_end on are left
    for the caller."""
    half = n // 2
    n_end = n if n_end is None else n_end
    x = np.empty(n, dtype=dtype)
    y = np.empty(n, dtype=dtype)
    x[:half] = np.ldexp(mx[:half], kx).astype(dtype)
    y[:half] = np.ldexp(my[:half], ky).astype(dtype)
    mxt = np.ascontiguousarray(mx[half:n_end], dtype=np.float64)
    myt = np.ascontiguousarray(my[half:n_end], dtype=np.float64)
    L = _clib()
    p_final = ctypes.c_double(0.0)
    if dtype == np.float64:
        tiny = 2.0 ** (-1022 + 53)
        small = L.synth_illcond_tail_f64(x.ctypes.data, y.ctypes.data, half, n_end,
                                         mxt.ctypes.data, myt.ctypes.data, h, tiny,
                                         ctypes.byref(p_final))
    else:
        tiny = 2.0 ** (-126 + 24)
        small = L.synth_illcond_tail_f32(x.ctypes.data, y.ctypes.data, half, n_end,
                                         mxt.ctypes.data, myt.ctypes.data, h, tiny,
                                         ctypes.byref(p_final))
    if small:
        raise ValueError("illcond_dot: %d products below the FMA-exactness range" % small)
    if not (np.all(np.isfinite(x[:n_end])) and np.all(np.isfinite(y[:n_end]))):
        raise ValueError("illcond_dot: non-finite value generated")
    return x, y, p_final.value


def _estimate_cond(x, y, p_final):
    a = float(np.sum(np.abs(x.astype(np.float64) * y.astype(np.float64))))
    return (2.0 * a / abs(p_final) if p_final != 0 else float("inf")), a


def illcond_dot(seed, n, cond, dtype, calibrate=True, low_block=True):
    """Ill-conditioned dot-product inputs of length n (even, >= 4).

    b = log2(cond), h = round(b / 2). First half: x_i = m * 2^k and
    y_i = m' * 2^k' with m, m' uniform(-1, 1) and k, k' uniform integers in
    [0, h]. Second half: x_i = m * 2^e_i, e_i decaying linearly from h to 0,
    and y_i chosen so the running dot cancels toward m' * 2^e_i (see
    illcond.c). Draw order: m_x (n), m_y (n), k_x (n/2), k_y (n/2).

    The recipe overshoots its target (the cancellation leaves a sum of
    order 1 while sum |x y| grows with n), so with ``calibrate`` the same
    draws are used once more with h lowered by
    round(log2(estimate / cond) / 2), the estimate being
    2 * sum|x y| (binary64) / |final running dot| (x87 extended, rounded).

    Even at h = 0 the recipe stays near n/2 or above (every cancelling step
    adds a term of the size of the running dot, so sum|x y| grows like n
    while the dot stays of order 1). For a lower target (``low_block``,
    when the calibrated estimate still exceeds cond by more than 10^0.5)
    the cancelling tail ends at n - n/16, and the last n/16 elements form a
    non-cancelling block: x_i = m_i (the same draws), y_i = c * s *
    sign(x_i) * |m'_i|, so every product has the sign s of the running dot
    and the block adds T = sum|x y| over it, c chosen so that
    2 (A + T) / (|P| + T) = cond, A and P being sum|x y| and the running
    dot before the block. The exact achieved condition must still be
    measured by the caller."""
    if n < 4 or n % 2:
        raise ValueError("illcond_dot: n must be even and >= 4")
    dtype = np.dtype(dtype)
    h = int(round(np.log2(float(cond)) / 2.0))
    half = n // 2
    rng = _rng(seed)
    mx = raw_to_uniform(raw(rng, n), dtype)
    my = raw_to_uniform(raw(rng, n), dtype)
    ux = raw(rng, half)
    uy = raw(rng, half)
    for attempt in range(2 if calibrate else 1):
        kx = raw_to_int(ux, 0, h).astype(np.int32)
        ky = raw_to_int(uy, 0, h).astype(np.int32)
        x, y, p_final = _illcond_once(mx, my, kx, ky, n, h, dtype)
        est, _ = _estimate_cond(x, y, p_final)
        if attempt == 0 and calibrate:
            delta = int(round(np.log2(est / float(cond)) / 2.0)) if np.isfinite(est) else 0
            if delta <= 0:
                break
            h = max(0, h - delta)
    if low_block and calibrate and est > float(cond) * 10 ** 0.5 and n >= 64:
        m = n // 16
        n_end = n - m
        x, y, p_ill = _illcond_once(mx, my, kx, ky, n, h, dtype, n_end=n_end)
        _, a_ill = _estimate_cond(x[:n_end], y[:n_end], 1.0)
        t = (2.0 * a_ill - float(cond) * abs(p_ill)) / (float(cond) - 2.0)
        if t > 0:
            s = 1.0 if p_ill >= 0 else -1.0
            xb = mx[n_end:].astype(dtype)
            base = np.abs(xb.astype(np.float64) * my[n_end:].astype(np.float64))
            c = t / float(np.sum(base)) if np.sum(base) > 0 else 0.0
            x[n_end:] = xb
            y[n_end:] = (s * c * np.sign(xb.astype(np.float64)) *
                         np.abs(my[n_end:].astype(np.float64))).astype(dtype)
        else:  # the cancelling part alone already meets the target
            x, y, _ = _illcond_once(mx, my, kx, ky, n, h, dtype)
    return x, y


def illcond_seed(decade):
    """Seed of the ill-conditioned inputs with target condition 10**decade."""
    return (4, int(decade))


def illcond_perm_seed(decade):
    """Seed of the permutation applied to those inputs (permuted variant)."""
    return (4, int(decade), 1)


def permute_pairs(seed, x, y):
    """x and y reordered by one seeded permutation: positions sorted by n
    raw 64-bit draws (stable sort, so ties, if any, keep index order). The
    multiset of products x_i*y_i, hence the exact dot and its condition, is
    unchanged; the running sums no longer cancel in order."""
    order = np.argsort(raw(_rng(seed), x.size), kind="stable")
    return np.ascontiguousarray(x[order]), np.ascontiguousarray(y[order])


def segment_lengths(seed, nseg, max_len=1 << 20):
    """nseg lengths log-uniform in [1, max_len]:
    L = max(1, floor(exp(u * ln(max_len)))) with u uniform in [0, 1)."""
    rng = _rng(seed)
    u = raw_to_unit(raw(rng, nseg))
    L = np.floor(np.exp(u * np.log(float(max_len)))).astype(np.int64)
    return np.maximum(L, 1)


def offsets_from_lengths(lengths):
    off = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(np.asarray(lengths, dtype=np.int64), out=off[1:])
    return off


def hundred_hours():
    """The counter of the paper's "100 hours" test: 3,600,000 ticks of
    binary32 0.1 (one tick per tenth of a second for 100 hours)."""
    return np.full(3_600_000, np.float32(0.1), dtype=np.float32)
