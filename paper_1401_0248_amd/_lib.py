"""ctypes declarations of libtwofold.so (include/twofold.h).

Argument marshalling only. If the library has not been built, it is built
here once; if it cannot be loaded, import fails loudly: there is no CPU
fallback for any entry point.
"""
import ctypes
import os

from . import build as _build

OK, EINVAL, EWORKSPACE, EHIP, EALIGN, EOFFSETS, ENOTUNED, ECAPTURE = 0, -1, -2, -3, -4, -5, -6, -7
PLAIN, FAST, RIGOROUS, WIDE, KAHAN, FAST_ROUNDED, RIGOROUS_ROUNDED, MIXED = 0, 1, 2, 3, 4, 5, 6, 7
FLAG_ERROR, FLAG_LENGTH, FLAG_NONFINITE = 1, 2, 4

# Every symbol the public header declares, with (restype, argtypes).
_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_int = ctypes.c_int
_sz = ctypes.c_size_t


class Launch(ctypes.Structure):
    """twofold_launch_t."""
    _fields_ = [("block_threads", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("tile_elems", ctypes.c_int64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_ if f != "reserved"}


_LP = ctypes.POINTER(Launch)

SIGNATURES = {
    "twofold_default_launch": (_int, [_int, _int, _int, _int, _i64, _i64, _LP]),
    "twofold_tuned_launch": (_int, [_int, _int, _int, _int, _i64, _i64, _LP]),
    "twofold_workspace_bytes_single": (_sz, [_int, _int, _int, _i64, _LP]),
    "twofold_workspace_bytes_seg": (_sz, [_int, _int, _int, _i64, _i64, _LP]),
    "twofold_sum_f32": (_int, [_vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_sum_f64": (_int, [_vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_dot_f32": (_int, [_vp, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_dot_f64": (_int, [_vp, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_sumd_f32": (_int, [_vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_dotd_f32": (_int, [_vp, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_sumd_f64": (_int, [_vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_dotd_f64": (_int, [_vp, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_sum_mixed_f32": (_int, [_vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_dot_mixed_f32": (_int, [_vp, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_workspace_bytes_multi": (_sz, [_int, _int, _int, _vp, _i64, _LP]),
    "twofold_multisum_f32": (_int, [_vp, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_multisum_f64": (_int, [_vp, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_multidot_f32": (_int, [_vp, _vp, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_multidot_f64": (_int, [_vp, _vp, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_multisumd_f32": (_int, [_vp, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_multisumd_f64": (_int, [_vp, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_multidotd_f32": (_int, [_vp, _vp, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_multidotd_f64": (_int, [_vp, _vp, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_multisum_mixed_f32": (_int, [_vp, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_multidot_mixed_f32": (_int, [_vp, _vp, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segsum_f32": (_int, [_vp, _i64, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segsum_f64": (_int, [_vp, _i64, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segdot_f32": (_int, [_vp, _vp, _i64, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segdot_f64": (_int, [_vp, _vp, _i64, _vp, _i64, _int, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segsumd_f32": (_int, [_vp, _i64, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segsumd_f64": (_int, [_vp, _i64, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segdotd_f32": (_int, [_vp, _vp, _i64, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segdotd_f64": (_int, [_vp, _vp, _i64, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segsum_mixed_f32": (_int, [_vp, _i64, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_segdot_mixed_f32": (_int, [_vp, _vp, _i64, _vp, _i64, _LP, _vp, _vp, _sz, _vp]),
    "twofold_seg_plan_create": (_int, [_vp, _i64, _int, _int, _int, _LP, ctypes.POINTER(_vp)]),
    "twofold_seg_plan_workspace_bytes": (_sz, [_vp]),
    "twofold_seg_plan_get_launch": (_int, [_vp, _LP]),
    "twofold_seg_plan_execute": (_int, [_vp, _vp, _vp, _vp, _vp, _sz, _vp]),
    "twofold_seg_plan_destroy": (_int, [_vp]),
    "twofold_monitor": (_int, [_int, _vp, _i64, _vp, _i64, ctypes.c_double, _vp, _vp, _vp]),
    "twofold_probe_read": (_int, [_vp, _vp, _i64, _LP, _vp, _vp]),
    "twofold_probe_compute": (_int, [_int, _int, _int, _vp, _i64, _LP, _vp, _vp]),
    "twofold_workspace_bytes_batch": (_sz, [_vp, _i64, _LP]),
    "twofold_batch": (_int, [_vp, _i64, _LP, _vp, _sz, _vp]),
    "twofold_batch_static": (_int, [_vp, _i64, _LP, _vp]),
    "twofold_strerror": (ctypes.c_char_p, [_int]),
}

class BatchItem(ctypes.Structure):
    """twofold_batch_item_t of include/twofold.h."""
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("out", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("dtype", ctypes.c_int32), ("is_dot", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lib = None


def lib_path():
    # TWOFOLD_HIP_LIB: another build of the library (the host-sanitizer
    # test's), used as is
    return os.environ.get("TWOFOLD_HIP_LIB") or _build.LIB


def load():
    """Load libtwofold.so (building it first if it does not exist)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if path == _build.LIB and not os.path.exists(path):
        _build.build()
    try:
        L = ctypes.CDLL(path)
    except OSError as exc:  # no silent fallback
        raise RuntimeError("cannot load the HIP library %s: %s" % (path, exc)) from exc
    for name, (res, args) in SIGNATURES.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


class TwofoldError(RuntimeError):
    def __init__(self, fn, status):
        msg = load().twofold_strerror(status).decode()
        super().__init__("%s failed: %s (%d)" % (fn, msg, status))
        self.status = status


def check(fn, status):
    if status != OK:
        raise TwofoldError(fn, status)
