"""Twofold summation on AMD Instinct MI355X (gfx950).

Python binding of libtwofold.so (include/twofold.h): each function checks
its tensors, takes the device pointers and torch's current HIP stream, and
calls the C entry point of the same name. All arithmetic runs in the HIP
kernels; torch only provides device memory and streams.

Results are device tensors holding (value, error) pairs (E. Latkin,
"Twofold fast summation": value is the plain floating-point sum, error the
collected round-offs; section "Algorithms").
"""
import ctypes

import torch

from . import _lib
from ._lib import (FAST, FAST_ROUNDED, FLAG_ERROR, FLAG_LENGTH, FLAG_NONFINITE, KAHAN, MIXED, PLAIN,
                   RIGOROUS, RIGOROUS_ROUNDED, WIDE, Launch, TwofoldError, check)

__all__ = [
    "sum", "dot", "sumd", "dotd", "sum_mixed", "dot_mixed", "multisum", "multidot", "segsum",
    "segdot", "SegPlan",
    "Launch", "monitor",
    "TwofoldError", "workspace", "default_launch", "tuned_launch", "probe_read", "probe_compute",
    "FLAG_ERROR", "FLAG_LENGTH", "FLAG_NONFINITE",
    "PLAIN", "FAST", "RIGOROUS", "WIDE", "KAHAN", "FAST_ROUNDED", "RIGOROUS_ROUNDED", "MIXED",
    "mode_id",
]

_MODES = {"plain": PLAIN, "fast": FAST, "rigorous": RIGOROUS, "wide": WIDE, "kahan": KAHAN,
          "fast_rounded": FAST_ROUNDED, "rigorous_rounded": RIGOROUS_ROUNDED, "mixed": MIXED}


def mode_id(mode):
    if isinstance(mode, str):
        return _MODES[mode]
    return int(mode)


def _launch_ptr(launch):
    if launch is None:
        return None
    if isinstance(launch, dict):
        launch = Launch(**launch)
    return ctypes.byref(launch)


def _stream_ptr(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _out(out, rows, dtype, device, shape):
    """The output tensor: a new one, or the caller's after checking that the
    library's rows fit it (the library writes rows pairs of dtype)."""
    if out is None:
        return torch.empty(shape, dtype=dtype, device=device)
    if not isinstance(out, torch.Tensor) or out.device != torch.device(device) or \
            out.dtype != dtype or not out.is_contiguous() or out.numel() < 2 * rows:
        raise ValueError("twofold: out must be a contiguous %s tensor of at least %d elements "
                         "on %s" % (dtype, 2 * rows, device))
    return out


def _check_data(*ts):
    t0 = ts[0]
    if not t0.is_cuda:
        raise ValueError("twofold: tensors must be on a GPU device")
    if t0.dtype not in (torch.float32, torch.float64):
        raise TypeError("twofold: dtype must be float32 or float64, got %s" % t0.dtype)
    for t in ts:
        if t.dim() != 1 or not t.is_contiguous():
            raise ValueError("twofold: tensors must be 1-D and contiguous")
        if t.dtype != t0.dtype or t.device != t0.device:
            raise ValueError("twofold: tensors must share dtype and device")
    if len(ts) == 2 and ts[0].numel() != ts[1].numel():
        raise ValueError("twofold: x and y must have the same length")


class Workspace:
    """Device scratch for the library's calls (no preparation needed)."""

    def __init__(self, nbytes, device):
        nbytes = max(256, int(nbytes))
        # 256-byte alignment: the caching allocator returns 512-byte blocks.
        self.buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        self.ptr = (self.buf.data_ptr() + 255) & ~255
        self.nbytes = nbytes


_ws_cache = {}


def workspace(nbytes, device):
    """The per-(device, stream) workspace, grown to at least nbytes. Calls on
    one stream run in order, so they can share it. (A graph captured on a
    stream keeps using the workspace it was captured with.)"""
    device = torch.device(device)
    stream = torch.cuda.current_stream(device).cuda_stream
    key = (device.index, stream)
    ws = _ws_cache.get(key)
    if ws is None or ws.nbytes < nbytes:
        ws = Workspace(max(nbytes, 2 * ws.nbytes if ws else nbytes), device)
        _ws_cache[key] = ws
    return ws


def default_launch(kind, dtype, is_dot, mode, n, nseg=0):
    lc = Launch()
    check("twofold_default_launch",
          _lib.load().twofold_default_launch(kind, dtype, int(is_dot), mode_id(mode), n, nseg,
                                             ctypes.byref(lc)))
    return lc


def tuned_launch(kind, dtype, is_dot, mode, n, nseg=0):
    """(launch, measured): the default launch, and whether the autotuner
    measured a row of its own for this configuration (twofold_tuned_launch;
    False when the default is borrowed from another mode or built in)."""
    lc = Launch()
    rc = _lib.load().twofold_tuned_launch(kind, dtype, int(is_dot), mode_id(mode), n, nseg,
                                          ctypes.byref(lc))
    if rc not in (_lib.OK, _lib.ENOTUNED):
        check("twofold_tuned_launch", rc)
    return lc, rc == _lib.OK


def _single(fn, x, y, mode, launch, out, ws, out_dtype):
    L = _lib.load()
    _check_data(*([x] if y is None else [x, y]))
    dev = x.device
    n = x.numel()
    dt = x.element_size()
    m = mode_id(mode)
    lp = _launch_ptr(launch)
    need = L.twofold_workspace_bytes_single(dt, int(y is not None), m, n, lp)
    if need == 0:
        raise TwofoldError("twofold_workspace_bytes_single", _lib.EINVAL)
    out = _out(out, 1, out_dtype, dev, (2,))
    if ws is None:
        ws = workspace(need, dev)
    args = [ctypes.c_void_p(x.data_ptr())]
    if y is not None:
        args.append(ctypes.c_void_p(y.data_ptr()))
    args.append(n)
    if not fn.startswith(("twofold_sumd_", "twofold_dotd_", "twofold_sum_mixed_",
                          "twofold_dot_mixed_")):
        args.append(m)
    args += [lp, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.ptr), ws.nbytes,
             _stream_ptr(dev)]
    check(fn, getattr(L, fn)(*args))
    return out


def sum(x, mode="rigorous", launch=None, out=None, ws=None):  # noqa: A001 (paper's name)
    """Twofold sum of x: tensor([value, error]) of x's dtype (Example 1 fast,
    Example 3 rigorous, or plain)."""
    fn = "twofold_sum_f32" if x.dtype == torch.float32 else "twofold_sum_f64"
    return _single(fn, x, None, mode, launch, out, ws, x.dtype)


def dot(x, y, mode="rigorous", launch=None, out=None, ws=None):
    """Twofold dot product of x and y: tensor([value, error])."""
    fn = "twofold_dot_f32" if x.dtype == torch.float32 else "twofold_dot_f64"
    return _single(fn, x, y, mode, launch, out, ws, x.dtype)


def sumd(x, launch=None, out=None, ws=None):
    """Paper's sumd, the wider accumulator: float32 data summed in float64;
    float64 data summed in double-word arithmetic (the paper used quad).
    Returns a float64 tensor([value, error])."""
    fn = "twofold_sumd_f32" if x.dtype == torch.float32 else "twofold_sumd_f64"
    return _single(fn, x, None, WIDE, launch, out, ws, torch.float64)


def dotd(x, y, launch=None, out=None, ws=None):
    """Paper's dotd: float32 data with float64 products and accumulator;
    float64 data with exact products in a double-word accumulator."""
    fn = "twofold_dotd_f32" if x.dtype == torch.float32 else "twofold_dotd_f64"
    return _single(fn, x, y, WIDE, launch, out, ws, torch.float64)


MAX_MULTI = 64  # vectors per multi-vector call


def _multi(fn, xs, ys, mode, launch, out, ws):
    L = _lib.load()
    xs = list(xs)
    ys = None if ys is None else list(ys)
    count = len(xs)
    if not 1 <= count <= MAX_MULTI:
        raise ValueError("twofold: a multi-vector call takes 1..%d vectors" % MAX_MULTI)
    if ys is not None and len(ys) != count:
        raise ValueError("twofold: xs and ys must have the same number of vectors")
    for v in range(count):
        _check_data(*([xs[v]] if ys is None else [xs[v], ys[v]]))
        if xs[v].dtype != xs[0].dtype or xs[v].device != xs[0].device:
            raise ValueError("twofold: all vectors must share dtype and device")
    dev = xs[0].device
    dt = xs[0].element_size()
    m = mode_id(mode)
    lp = _launch_ptr(launch)
    ns = (ctypes.c_int64 * count)(*[x.numel() for x in xs])
    xp = (ctypes.c_void_p * count)(*[x.data_ptr() for x in xs])
    need = L.twofold_workspace_bytes_multi(dt, int(ys is not None), m, ctypes.cast(ns, ctypes.c_void_p),
                                           count, lp)
    if need == 0:
        raise TwofoldError("twofold_workspace_bytes_multi", _lib.EINVAL)
    odt = torch.float64 if m in (WIDE, MIXED) else xs[0].dtype
    out = _out(out, count, odt, dev, (count, 2))
    if ws is None:
        ws = workspace(need, dev)
    args = [ctypes.cast(xp, ctypes.c_void_p)]
    if ys is not None:
        yp = (ctypes.c_void_p * count)(*[y.data_ptr() for y in ys])
        args.append(ctypes.cast(yp, ctypes.c_void_p))
    args.append(ctypes.cast(ns, ctypes.c_void_p))
    args.append(count)
    if not fn.startswith(("twofold_multisumd_", "twofold_multidotd_", "twofold_multisum_mixed_",
                          "twofold_multidot_mixed_")):
        args.append(m)
    args += [lp, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.ptr), ws.nbytes,
             _stream_ptr(dev)]
    check(fn, getattr(L, fn)(*args))
    return out


def multisum(xs, mode="rigorous", launch=None, out=None, ws=None):
    """Twofold sums of up to 64 vectors in one launch: a (count, 2) tensor,
    row v bitwise the sum() of xs[v] with the same launch (default: the
    launch of the longest vector)."""
    fn = "twofold_multisum_f32" if xs[0].dtype == torch.float32 else "twofold_multisum_f64"
    return _multi(fn, xs, None, mode, launch, out, ws)


def multidot(xs, ys, mode="rigorous", launch=None, out=None, ws=None):
    """Twofold dots of up to 64 vector pairs in one launch: a (count, 2)
    tensor, row v bitwise the dot() of (xs[v], ys[v]) with the same launch."""
    fn = "twofold_multidot_f32" if xs[0].dtype == torch.float32 else "twofold_multidot_f64"
    return _multi(fn, xs, ys, mode, launch, out, ws)


def multisumd(xs, launch=None, out=None, ws=None):
    """sumd() of up to 64 vectors in one launch: a (count, 2) float64
    tensor, row v bitwise sumd(xs[v]) with the same launch."""
    fn = "twofold_multisumd_f32" if xs[0].dtype == torch.float32 else "twofold_multisumd_f64"
    return _multi(fn, xs, None, WIDE, launch, out, ws)


def multidotd(xs, ys, launch=None, out=None, ws=None):
    """dotd() of up to 64 vector pairs in one launch (float64 rows)."""
    fn = "twofold_multidotd_f32" if xs[0].dtype == torch.float32 else "twofold_multidotd_f64"
    return _multi(fn, xs, ys, WIDE, launch, out, ws)


def multisum_mixed(xs, launch=None, out=None, ws=None):
    """sum_mixed() of up to 64 float32 vectors in one launch (float64 rows)."""
    if xs[0].dtype != torch.float32:
        raise TypeError("twofold: the mixed form takes float32 data")
    return _multi("twofold_multisum_mixed_f32", xs, None, MIXED, launch, out, ws)


def multidot_mixed(xs, ys, launch=None, out=None, ws=None):
    """dot_mixed() of up to 64 float32 vector pairs in one launch."""
    if xs[0].dtype != torch.float32:
        raise TypeError("twofold: the mixed form takes float32 data")
    return _multi("twofold_multidot_mixed_f32", xs, ys, MIXED, launch, out, ws)


MAX_BATCH = 64  # items per batch call


def batch(items, launch=None, outs=None, ws=None):
    """Up to 64 sums and dots of either data type and any mode in one launch
    (twofold_batch). items: (x, y, mode) tuples, y None for a sum. Returns
    one tensor([value, error]) per item (float64 for "wide" and "mixed"),
    bitwise that item's single call (sum/dot, sumd/dotd, sum_mixed/dot_mixed)
    with the batch's launch (default: the launch of the item that reads the
    most bytes, at most four vectors a round when its blocks have more than
    512 threads)."""
    L = _lib.load()
    arr, count, res, dev = _batch_items(items, outs)
    lp = _launch_ptr(launch)
    need = L.twofold_workspace_bytes_batch(ctypes.cast(arr, ctypes.c_void_p), count, lp)
    if need == 0:
        raise TwofoldError("twofold_workspace_bytes_batch", _lib.EINVAL)
    if ws is None:
        ws = workspace(need, dev)
    check("twofold_batch", L.twofold_batch(ctypes.cast(arr, ctypes.c_void_p), count, lp,
                                           ctypes.c_void_p(ws.ptr), ws.nbytes, _stream_ptr(dev)))
    return res


def batch_static(items, launch=None, outs=None):
    """batch() without a workspace (twofold_batch_static): the block pairs
    go to the library's static per-device scratch of 4 MiB, so the call
    allocates nothing (torch included, when outs are given). Calls that can
    overlap on one device race on that scratch."""
    L = _lib.load()
    arr, count, res, dev = _batch_items(items, outs)
    check("twofold_batch_static", L.twofold_batch_static(
        ctypes.cast(arr, ctypes.c_void_p), count, _launch_ptr(launch), _stream_ptr(dev)))
    return res


def _batch_items(items, outs):
    """The twofold_batch_item_t array of a batch, and its output tensors."""
    items = list(items)
    count = len(items)
    if not 1 <= count <= MAX_BATCH:
        raise ValueError("twofold: a batch takes 1..%d items" % MAX_BATCH)
    if outs is not None and len(outs) != count:
        raise ValueError("twofold: one out per item")
    dev = items[0][0].device
    arr = (_lib.BatchItem * count)()
    res = []
    for v, (x, y, mode) in enumerate(items):
        _check_data(*([x] if y is None else [x, y]))
        if x.device != dev:
            raise ValueError("twofold: all items must be on one device")
        m = mode_id(mode)
        odt = torch.float64 if m in (WIDE, MIXED) else x.dtype
        o = _out(None if outs is None else outs[v], 1, odt, dev, (2,))
        res.append(o)
        arr[v].x = x.data_ptr()
        arr[v].y = y.data_ptr() if y is not None else None
        arr[v].out = o.data_ptr()
        arr[v].n = x.numel()
        arr[v].dtype = x.element_size()
        arr[v].is_dot = int(y is not None)
        arr[v].mode = m
    return arr, count, res, dev


def sum_mixed(x, launch=None, out=None, ws=None):
    """Rigorous twofold sum of float32 data with a float64 error term: a
    float64 tensor([value, error]) whose value is sum(x, "rigorous")'s."""
    if x.dtype != torch.float32:
        raise TypeError("twofold: the mixed form takes float32 data")
    return _single("twofold_sum_mixed_f32", x, None, MIXED, launch, out, ws, torch.float64)


def dot_mixed(x, y, launch=None, out=None, ws=None):
    """Rigorous twofold dot of float32 data with a float64 error term."""
    if x.dtype != torch.float32:
        raise TypeError("twofold: the mixed form takes float32 data")
    return _single("twofold_dot_mixed_f32", x, y, MIXED, launch, out, ws, torch.float64)


def _seg(x, y, offsets, mode, launch, out, ws, fn=None):
    L = _lib.load()
    _check_data(*([x] if y is None else [x, y]))
    if offsets.dtype != torch.int64 or offsets.device != x.device or offsets.dim() != 1 \
            or not offsets.is_contiguous():
        raise ValueError("twofold: offsets must be a contiguous int64 tensor on x's device")
    nseg = offsets.numel() - 1
    if nseg < 0:
        raise ValueError("twofold: offsets must hold nseg + 1 entries")
    dev = x.device
    dt = x.element_size()
    m = mode_id(mode)
    lp = _launch_ptr(launch)
    n_total = x.numel()
    need = L.twofold_workspace_bytes_seg(dt, int(y is not None), m, n_total, nseg, lp)
    if need == 0:
        raise TwofoldError("twofold_workspace_bytes_seg", _lib.EINVAL)
    odt = torch.float64 if (fn is not None or x.dtype == torch.float64) else x.dtype
    out = _out(out, nseg, odt, dev, (nseg, 2))
    if ws is None:
        ws = workspace(need, dev)
    sfx = "f32" if x.dtype == torch.float32 else "f64"
    if fn is None:  # the generic calls take the mode
        fn = ("twofold_segsum_" if y is None else "twofold_segdot_") + sfx
        tail = [m, lp]
    else:
        tail = [lp]
    args = [ctypes.c_void_p(x.data_ptr())]
    if y is not None:
        args.append(ctypes.c_void_p(y.data_ptr()))
    args += [n_total, ctypes.c_void_p(offsets.data_ptr()), nseg] + tail + \
        [ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.ptr), ws.nbytes, _stream_ptr(dev)]
    check(fn, getattr(L, fn)(*args))
    return out


def segsum(x, offsets, mode="rigorous", launch=None, out=None, ws=None):
    """Twofold sums of the CSR segments of x: (nseg, 2) tensor."""
    return _seg(x, None, offsets, mode, launch, out, ws)


def segdot(x, y, offsets, mode="rigorous", launch=None, out=None, ws=None):
    """Twofold dot products of the CSR segments of x and y: (nseg, 2)."""
    return _seg(x, y, offsets, mode, launch, out, ws)


def segsumd(x, offsets, launch=None, out=None, ws=None):
    """sumd() of every CSR segment of x: (nseg, 2) float64 rows."""
    fn = "twofold_segsumd_f32" if x.dtype == torch.float32 else "twofold_segsumd_f64"
    return _seg(x, None, offsets, WIDE, launch, out, ws, fn)


def segdotd(x, y, offsets, launch=None, out=None, ws=None):
    """dotd() of every CSR segment of x and y: (nseg, 2) float64 rows."""
    fn = "twofold_segdotd_f32" if x.dtype == torch.float32 else "twofold_segdotd_f64"
    return _seg(x, y, offsets, WIDE, launch, out, ws, fn)


def segsum_mixed(x, offsets, launch=None, out=None, ws=None):
    """sum_mixed() of every CSR segment of float32 x: (nseg, 2) float64 rows."""
    if x.dtype != torch.float32:
        raise TypeError("twofold: the mixed form takes float32 data")
    return _seg(x, None, offsets, MIXED, launch, out, ws, "twofold_segsum_mixed_f32")


def segdot_mixed(x, y, offsets, launch=None, out=None, ws=None):
    """dot_mixed() of every CSR segment of float32 x and y (float64 rows)."""
    if x.dtype != torch.float32:
        raise TypeError("twofold: the mixed form takes float32 data")
    return _seg(x, y, offsets, MIXED, launch, out, ws, "twofold_segdot_mixed_f32")


class SegPlan:
    """A segmented reduction with host offsets fixed at creation; execute()
    is one persistent kernel and may be captured into a HIP graph."""

    def __init__(self, offsets_host, dtype, is_dot, mode="rigorous", launch=None):
        import numpy as np
        off = np.ascontiguousarray(offsets_host, dtype=np.int64)
        self.nseg = off.size - 1
        self.dtype = {torch.float32: 4, torch.float64: 8}.get(dtype, dtype)
        self.is_dot = bool(is_dot)
        self.mode = mode_id(mode)
        self._L = _lib.load()
        h = ctypes.c_void_p()
        check("twofold_seg_plan_create", self._L.twofold_seg_plan_create(
            ctypes.c_void_p(off.ctypes.data), self.nseg, self.dtype, int(self.is_dot), self.mode,
            _launch_ptr(launch), ctypes.byref(h)))
        self._h = h
        self.workspace_bytes = self._L.twofold_seg_plan_workspace_bytes(h)
        self.launch = Launch()
        check("twofold_seg_plan_get_launch",
              self._L.twofold_seg_plan_get_launch(h, ctypes.byref(self.launch)))

    @property
    def out_dtype(self):
        return torch.float64 if (self.dtype == 8 or self.mode in (WIDE, MIXED)) else torch.float32

    def execute(self, x, y=None, out=None, ws=None):
        _check_data(*([x] if y is None else [x, y]))
        if x.element_size() != self.dtype:
            raise TypeError("SegPlan: data type differs from the plan's")
        out = _out(out, self.nseg, self.out_dtype, x.device, (self.nseg, 2))
        if ws is None:
            ws = workspace(self.workspace_bytes, x.device)
        if self.is_dot != (y is not None):
            raise ValueError("SegPlan: y must be given exactly for dot plans")
        check("twofold_seg_plan_execute", self._L.twofold_seg_plan_execute(
            self._h, ctypes.c_void_p(x.data_ptr()),
            ctypes.c_void_p(y.data_ptr()) if y is not None else None,
            ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.ptr), ws.nbytes,
            _stream_ptr(x.device)))
        return out

    def close(self):
        if getattr(self, "_h", None):
            check("twofold_seg_plan_destroy", self._L.twofold_seg_plan_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def monitor(pairs, tau, offsets=None, n=None, flags=None, nflagged=None):
    """Precision monitor (twofold_monitor): pairs is a (count, 2) float32 or
    float64 device tensor of (value, error) results, e.g. a segmented
    call's output; lengths come from offsets (device int64, count + 1
    entries) or are all n. Returns (flags, nflagged): uint32-valued flags
    (stored as int32) per result and the count of flagged results (int64
    device scalar), both on the device."""
    L = _lib.load()
    if not pairs.is_cuda or pairs.dtype not in (torch.float32, torch.float64) or \
            pairs.dim() != 2 or pairs.shape[1] != 2 or not pairs.is_contiguous():
        raise ValueError("pairs must be a contiguous (count, 2) float32 or float64 GPU tensor")
    if offsets is None and n is None:
        raise ValueError("give offsets or n")
    dev = pairs.device
    count = pairs.shape[0]
    if offsets is not None:
        if offsets.dtype != torch.int64 or offsets.dim() != 1 or not offsets.is_contiguous() or \
                offsets.numel() != count + 1 or offsets.device != dev:
            raise ValueError("offsets must be a contiguous int64 tensor of count + 1 entries on "
                             "the pairs' device")
    if flags is None:
        flags = torch.empty(count, dtype=torch.int32, device=dev)
    elif flags.device != dev or flags.element_size() != 4 or not flags.is_contiguous() or \
            flags.numel() < count:
        raise ValueError("flags must be a contiguous 4-byte tensor of count entries on the "
                         "pairs' device")
    if nflagged is None:
        nflagged = torch.empty((), dtype=torch.int64, device=dev)
    elif nflagged.device != dev or nflagged.dtype != torch.int64 or nflagged.numel() < 1:
        raise ValueError("nflagged must be an int64 tensor on the pairs' device")
    check("twofold_monitor", L.twofold_monitor(
        pairs.element_size(), ctypes.c_void_p(pairs.data_ptr()) if count else None, count,
        ctypes.c_void_p(offsets.data_ptr()) if offsets is not None else None,
        0 if n is None else int(n), float(tau),
        ctypes.c_void_p(flags.data_ptr()) if count else None, ctypes.c_void_p(nflagged.data_ptr()),
        _stream_ptr(dev)))
    return flags, nflagged


def probe_read(x, y=None, launch=None, sink=None):
    """Memory-only probe over the bytes of x (and y)."""
    L = _lib.load()
    if launch is None:
        launch = Launch(256, 4, 2048, 0, 0)
    elif isinstance(launch, dict):
        launch = Launch(**launch)
    nbytes = x.numel() * x.element_size()
    if sink is None:
        sink = torch.empty(launch.grid_blocks, dtype=torch.int64, device=x.device)
    elif sink.device != x.device or sink.element_size() != 8 or not sink.is_contiguous() or \
            sink.numel() < launch.grid_blocks:
        raise ValueError("sink must be a contiguous 8-byte tensor of grid_blocks entries")
    check("twofold_probe_read", L.twofold_probe_read(
        ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()) if y is not None else None,
        nbytes, ctypes.byref(launch), ctypes.c_void_p(sink.data_ptr()), _stream_ptr(x.device)))
    return sink


def probe_compute(seed, is_dot, mode, iters, launch, sink=None):
    """Compute-only probe; seed: 64 values of the data type on the device."""
    L = _lib.load()
    if isinstance(launch, dict):
        launch = Launch(**launch)
    if not seed.is_cuda or seed.dtype not in (torch.float32, torch.float64) or \
            not seed.is_contiguous() or seed.numel() < 64:
        raise ValueError("seed must be a contiguous float32 or float64 GPU tensor of 64 values")
    need = 2 * launch.grid_blocks * launch.block_threads
    if sink is None:
        sink = torch.empty(need, dtype=torch.float64, device=seed.device)
    elif sink.device != seed.device or sink.element_size() != 8 or not sink.is_contiguous() or \
            sink.numel() < need:
        raise ValueError("sink must be a contiguous 8-byte tensor of 2 * grid_blocks * "
                         "block_threads entries")
    check("twofold_probe_compute", L.twofold_probe_compute(
        seed.element_size(), int(is_dot), mode_id(mode), ctypes.c_void_p(seed.data_ptr()), iters,
        ctypes.byref(launch), ctypes.c_void_p(sink.data_ptr()), _stream_ptr(seed.device)))
    return sink
