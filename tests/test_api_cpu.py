"""The C interface without a GPU: the library loads, exports every function
include/twofold.h declares, and rejects bad arguments on the host before
any HIP call (so these calls are safe on a machine with no GPU)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_1401_0248_amd import _lib
from paper_1401_0248_amd._lib import EALIGN, EINVAL, EOFFSETS, EWORKSPACE, Launch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "twofold.h")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(twofold_\w+)\s*\(", txt)))


def test_every_declared_symbol_is_exported():
    L = _lib.load()
    names = _declared()
    assert len(names) >= 20
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.lib_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (twofold_\w+)", out))
    for n in names:
        assert n in exported, n
        assert hasattr(L, n)
    # and the binding declares a signature for each of them
    assert set(names) == set(_lib.SIGNATURES)


def test_product_does_not_touch_the_oracle():
    out = subprocess.run(["nm", "-D", _lib.lib_path()], capture_output=True, text=True).stdout
    assert "oracle" not in out
    pkg = os.path.join(ROOT, "paper_1401_0248_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".inc", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "twofold_oracle" not in src, f


def test_header_compiles_as_c():
    src = '#include "twofold.h"\nint main(void){ twofold_launch_t l = {0}; (void)l; return 0; }\n'
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                        "-x", "c", "-", "-fsyntax-only"], input=src, text=True, capture_output=True)
    assert r.returncode == 0, r.stderr


def test_strerror():
    L = _lib.load()
    for code in (0, -1, -2, -3, -4, -5, 7):
        assert isinstance(L.twofold_strerror(code), bytes)


def test_single_argument_checks():
    L = _lib.load()
    fake = ctypes.c_void_p(0x10000)  # never dereferenced: checks fail first
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 20
    # null pointers, negative n, bad modes
    assert L.twofold_sum_f32(None, 10, 2, None, fake, ws, big, None) == EINVAL
    assert L.twofold_sum_f32(fake, -1, 2, None, fake, ws, big, None) == EINVAL
    assert L.twofold_sum_f32(fake, 10, 9, None, fake, ws, big, None) == EINVAL  # no such mode
    assert L.twofold_sum_f32(fake, 10, 3, None, fake, ws, big, None) == EINVAL  # wide: use sumd
    assert L.twofold_sum_f64(fake, 10, 3, None, fake, ws, big, None) == EINVAL  # wide: use sumd
    assert L.twofold_dot_f64(fake, fake, 10, 3, None, fake, ws, big, None) == EINVAL
    assert L.twofold_sum_f32(fake, 10, 5, None, fake, ws, big, None) == EINVAL  # rounded: dots only
    assert L.twofold_sum_f64(fake, 10, 6, None, fake, ws, big, None) == EINVAL
    assert L.twofold_sum_f64(fake, 10, 8, None, fake, ws, big, None) == EINVAL
    assert L.twofold_workspace_bytes_single(4, 0, 5, 100, None) == 0
    assert L.twofold_workspace_bytes_single(4, 1, 5, 100, None) > 0
    assert L.twofold_dot_f64(fake, None, 10, 2, None, fake, ws, big, None) == EINVAL
    # counts beyond 2^56
    assert L.twofold_sum_f32(fake, (1 << 56) + 1, 2, None, fake, ws, big, None) == EINVAL
    assert L.twofold_workspace_bytes_single(4, 0, 2, (1 << 63) - 1, None) == 0
    assert L.twofold_default_launch(0, 8, 1, 2, (1 << 63) - 1, 0, ctypes.byref(Launch())) == EINVAL
    # misaligned data
    assert L.twofold_sum_f64(ctypes.c_void_p(0x10004), 10, 2, None, fake, ws, big, None) == EALIGN
    assert L.twofold_dot_f32(fake, ctypes.c_void_p(0x10002), 10, 2, None, fake, ws, big, None) == EALIGN
    # workspace missing, misaligned, too small (needed once there are two blocks)
    many = Launch(256, 4, 5, 0, 0)
    assert L.twofold_sum_f32(fake, 10, 2, ctypes.byref(many), fake, None, big, None) == EWORKSPACE
    assert L.twofold_sum_f32(fake, 10, 2, ctypes.byref(many), fake, ctypes.c_void_p(0x100010), big,
                             None) == EWORKSPACE
    assert L.twofold_sum_f32(fake, 1 << 24, 2, None, fake, ws, 512, None) == EWORKSPACE
    # bad launches
    for lc in (Launch(100, 4, 1, 0, 0), Launch(256, 3, 1, 0, 0), Launch(256, 4, -1, 0, 0),
               Launch(256, 4, 1, 1, 0), Launch(32, 4, 1, 0, 0), Launch(2048, 4, 1, 0, 0),
               Launch(256, 4, (1 << 20) + 1, 0, 0)):
        assert L.twofold_sum_f32(fake, 10, 2, ctypes.byref(lc), fake, ws, big, None) == EINVAL


def test_workspace_sizes():
    L = _lib.load()
    for dt in (4, 8):
        for dot in (0, 1):
            b = L.twofold_workspace_bytes_single(dt, dot, 2, 1 << 24, None)
            lc = Launch()
            assert L.twofold_default_launch(0, dt, dot, 2, 1 << 24, 0, ctypes.byref(lc)) == 0
            assert b == ((16 * lc.grid_blocks + 255) // 256) * 256
            assert L.twofold_workspace_bytes_single(dt, dot, 2, 0, None) >= 16
    lc = Launch(256, 4, 7, 0, 0)
    assert L.twofold_workspace_bytes_single(8, 1, 2, 100, ctypes.byref(lc)) == 256
    # explicit grid is used as given
    assert L.twofold_default_launch(0, 8, 1, 2, 0, 0, ctypes.byref(lc)) == 0 and lc.grid_blocks == 1
    assert L.twofold_workspace_bytes_single(16, 1, 2, 100, None) == 0
    s = L.twofold_workspace_bytes_seg(4, 1, 2, 1 << 20, 1000, None)
    assert s > 256 + 8 * 1001 + 16 * 1000


def test_default_launch_grid_scales_with_n():
    L = _lib.load()
    lc = Launch()
    grids = []
    for n in (0, 1000, 1 << 16, 1 << 20, 1 << 28):
        assert L.twofold_default_launch(0, 4, 0, 2, n, 0, ctypes.byref(lc)) == 0
        grids.append(lc.grid_blocks)
        assert lc.block_threads % 64 == 0 and lc.unroll in (1, 2, 4, 8)
    assert grids[0] == 1 and grids == sorted(grids) and grids[-1] > 1


def test_segmented_argument_checks():
    L = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    ws = ctypes.c_void_p(0x100000)
    assert L.twofold_segsum_f32(fake, 10, None, 3, 2, None, fake, ws, 1 << 20, None) == EINVAL
    assert L.twofold_segsum_f32(fake, 10, fake, -1, 2, None, fake, ws, 1 << 20, None) == EINVAL
    assert L.twofold_segsum_f32(fake, 10, fake, 3, 3, None, fake, ws, 1 << 20, None) == EINVAL
    assert L.twofold_segsum_f64(fake, 10, ctypes.c_void_p(0x10004), 3, 2, None, fake, ws, 1 << 20,
                                None) == EALIGN
    assert L.twofold_segdot_f64(fake, fake, 1 << 20, fake, 5000, 2, None, fake, ws, 1024, None) == EWORKSPACE
    lc = Launch(256, 4, 16, 0, 1000)  # tile not a multiple of 64*W
    assert L.twofold_segsum_f32(fake, 10, fake, 3, 2, ctypes.byref(lc), fake, ws, 1 << 20, None) == EINVAL
    # a tile holds at most 2^30 elements (the tile kernel keeps a tile's
    # geometry in 32 bits), on both segmented paths
    big_tile = Launch(256, 4, 16, 0, (1 << 30) + 256)
    assert L.twofold_segsum_f32(fake, 10, fake, 3, 2, ctypes.byref(big_tile), fake, ws, 1 << 20,
                                None) == EINVAL
    offs = np.array([0, 4, 8, 10], dtype=np.int64)
    h = ctypes.c_void_p()
    assert L.twofold_seg_plan_create(offs.ctypes.data_as(ctypes.c_void_p), 3, 4, 0, 2,
                                     ctypes.byref(big_tile), ctypes.byref(h)) == EINVAL
    assert not h.value
    # nseg == 0: nothing to do, nothing launched
    assert L.twofold_segsum_f32(fake, 0, fake, 0, 2, None, fake, ws, 1 << 20, None) == 0
    # binary64 rows of binary32 data: their own calls, checked the same way
    assert L.twofold_segdot_f32(fake, fake, 10, fake, 3, 7, None, fake, ws, 1 << 20, None) == EINVAL
    assert L.twofold_segsumd_f32(fake, 10, None, 3, None, fake, ws, 1 << 20, None) == EINVAL
    assert L.twofold_segdot_mixed_f32(fake, None, 10, fake, 3, None, fake, ws, 1 << 20,
                                      None) == EINVAL
    assert L.twofold_segsum_mixed_f32(fake, 10, fake, 3, None, ctypes.c_void_p(0x10004), ws,
                                      1 << 20, None) == EALIGN  # binary64 output pairs
    assert L.twofold_segdotd_f64(fake, fake, 1 << 20, fake, 5000, None, fake, ws, 1024,
                                 None) == EWORKSPACE
    assert L.twofold_segsumd_f64(fake, 0, fake, 0, None, fake, ws, 1 << 20, None) == 0


def test_plan_rejects_bad_offsets_before_any_hip_call():
    L = _lib.load()
    h = ctypes.c_void_p()
    for off in ([1, 5, 9], [0, 5, 3], [0, -1]):
        a = np.array(off, dtype=np.int64)
        assert L.twofold_seg_plan_create(ctypes.c_void_p(a.ctypes.data), a.size - 1, 4, 0, 2, None,
                                         ctypes.byref(h)) == EOFFSETS
        assert not h.value
    a = np.array([0, 5], dtype=np.int64)
    assert L.twofold_seg_plan_create(ctypes.c_void_p(a.ctypes.data), 1, 8, 0, 5, None,
                                     ctypes.byref(h)) == EINVAL  # rounded forms: dots only
    assert L.twofold_seg_plan_create(ctypes.c_void_p(a.ctypes.data), 1, 8, 1, 9, None,
                                     ctypes.byref(h)) == EINVAL  # no such mode
    assert L.twofold_seg_plan_create(ctypes.c_void_p(a.ctypes.data), 1, 8, 1, 7, None,
                                     ctypes.byref(h)) == EINVAL  # mixed: binary32 only
    assert L.twofold_seg_plan_create(None, 1, 4, 0, 2, None, ctypes.byref(h)) == EINVAL
    a = np.array([0, 1 << 60], dtype=np.int64)
    assert L.twofold_seg_plan_create(ctypes.c_void_p(a.ctypes.data), 1, 4, 0, 2, None,
                                     ctypes.byref(h)) == EINVAL  # beyond 2^56 elements
    assert L.twofold_workspace_bytes_seg(4, 1, 2, 1 << 60, 10, None) == 0
    assert L.twofold_seg_plan_destroy(None) == 0
    assert L.twofold_seg_plan_workspace_bytes(None) == 0


def test_probe_argument_checks():
    L = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    lc = Launch(256, 4, 8, 0, 0)
    assert L.twofold_probe_read(fake, None, 100, ctypes.byref(lc), fake, None) == EINVAL
    assert L.twofold_probe_read(ctypes.c_void_p(0x10008), None, 160, ctypes.byref(lc), fake,
                                None) == EALIGN
    assert L.twofold_probe_read(fake, None, 160, None, fake, None) == EINVAL
    assert L.twofold_probe_compute(8, 0, 5, fake, 10, ctypes.byref(lc), fake, None) == EINVAL
    assert L.twofold_probe_compute(8, 1, 9, fake, 10, ctypes.byref(lc), fake, None) == EINVAL
    assert L.twofold_probe_compute(8, 1, 7, fake, 10, ctypes.byref(lc), fake, None) == EINVAL




def test_multi_argument_checks():
    L = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    ws = ctypes.c_void_p(0x100000)
    P = ctypes.c_void_p * 3
    N = ctypes.c_int64 * 3
    xs, ys, ns = P(0x10000, 0x20000, 0x30000), P(0x40000, 0x50000, 0x60000), N(10, 0, 7)
    big = 1 << 20
    assert L.twofold_multidot_f64(xs, ys, ns, 65, 2, None, fake, ws, big, None) == EINVAL
    assert L.twofold_multidot_f64(xs, ys, ns, -1, 2, None, fake, ws, big, None) == EINVAL
    assert L.twofold_multidot_f64(None, ys, ns, 3, 2, None, fake, ws, big, None) == EINVAL
    assert L.twofold_multidot_f64(xs, None, ns, 3, 2, None, fake, ws, big, None) == EINVAL
    assert L.twofold_multidot_f64(xs, ys, None, 3, 2, None, fake, ws, big, None) == EINVAL
    assert L.twofold_multidot_f64(xs, ys, ns, 3, 3, None, fake, ws, big, None) == EINVAL  # wide
    assert L.twofold_multisum_f32(xs, ns, 3, 5, None, fake, ws, big, None) == EINVAL  # rounded
    assert L.twofold_multisum_f32(xs, ns, 3, 2, None, None, ws, big, None) == EINVAL
    # count 0: nothing to do, nothing launched
    assert L.twofold_multisum_f32(None, None, 0, 2, None, fake, ws, big, None) == 0
    # a null data pointer only for an empty vector
    assert L.twofold_multisum_f64(P(0, 0x20000, 0x30000), ns, 3, 2, None, fake, ws, big,
                                  None) == EINVAL
    # misaligned data, too many elements
    assert L.twofold_multisum_f64(P(0x10000, 0x20000, 0x30004), ns, 3, 2, None, fake, ws, big,
                                  None) == EALIGN
    assert L.twofold_multidot_f32(xs, P(0x40000, 0x50002, 0x60000), ns, 3, 2, None, fake, ws,
                                  big, None) == EALIGN
    assert L.twofold_multisum_f32(xs, N(10, (1 << 56) + 1, 7), 3, 2, None, fake, ws, big,
                                  None) == EINVAL
    # workspace: count times the single-vector one of the longest vector's launch
    long_ns = N(1 << 24, 5, 1 << 20)
    one = L.twofold_workspace_bytes_single(8, 1, 2, 1 << 24, None)
    three = L.twofold_workspace_bytes_multi(8, 1, 2, long_ns, 3, None)
    assert one > 256 and three >= 3 * (one - 255)
    assert L.twofold_multidot_f64(xs, ys, long_ns, 3, 2, None, fake, ws, three - 256, None) == \
        EWORKSPACE
    assert L.twofold_workspace_bytes_multi(8, 1, 2, long_ns, 65, None) == 0
    # the wider accumulator and the mixed form: calls of their own, binary64 rows
    assert L.twofold_workspace_bytes_multi(8, 1, 3, long_ns, 3, None) >= 3 * 256  # double-word
    assert L.twofold_workspace_bytes_multi(4, 0, 7, long_ns, 3, None) >= 3 * 256
    assert L.twofold_workspace_bytes_multi(8, 0, 7, long_ns, 3, None) == 0  # mixed: binary32 only
    assert L.twofold_multisum_f32(xs, ns, 3, 7, None, fake, ws, big, None) == EINVAL
    assert L.twofold_multisum_f32(xs, ns, 3, 3, None, fake, ws, big, None) == EINVAL
    assert L.twofold_multisumd_f32(xs, ns, 3, None, ctypes.c_void_p(0x10004), ws, big,
                                   None) == EALIGN  # binary64 rows
    assert L.twofold_multidot_mixed_f32(xs, None, ns, 3, None, fake, ws, big, None) == EINVAL
    assert L.twofold_multidotd_f64(xs, ys, ns, 65, None, fake, ws, big, None) == EINVAL
    assert L.twofold_multisum_mixed_f32(None, None, 0, None, fake, ws, big, None) == 0
    assert L.twofold_multidotd_f32(xs, ys, long_ns, 3, None, fake, ws,
                                   L.twofold_workspace_bytes_multi(4, 1, 3, long_ns, 3, None) - 256,
                                   None) == EWORKSPACE


def test_mixed_mode_argument_checks():
    """The mixed form (mode 7) exists for binary32 data only and returns
    binary64 pairs: only twofold_{sum,dot}_mixed_f32, their multi-vector
    forms and plans take it."""
    L = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    ws = ctypes.c_void_p(0x100000)
    big = 1 << 20
    assert L.twofold_sum_f32(fake, 10, 7, None, fake, ws, big, None) == EINVAL
    assert L.twofold_dot_f32(fake, fake, 10, 7, None, fake, ws, big, None) == EINVAL
    assert L.twofold_sum_f64(fake, 10, 7, None, fake, ws, big, None) == EINVAL
    assert L.twofold_dot_f64(fake, fake, 10, 7, None, fake, ws, big, None) == EINVAL
    assert L.twofold_segsum_f32(fake, 10, fake, 3, 7, None, fake, ws, big, None) == EINVAL
    P = ctypes.c_void_p * 1
    N1 = ctypes.c_int64 * 1
    assert L.twofold_multisum_f32(P(0x10000), N1(10), 1, 7, None, fake, ws, big, None) == EINVAL
    assert L.twofold_workspace_bytes_multi(4, 0, 7, N1(10), 1, None) > 0
    assert L.twofold_workspace_bytes_multi(8, 0, 7, N1(10), 1, None) == 0
    assert L.twofold_workspace_bytes_single(8, 0, 7, 100, None) == 0
    assert L.twofold_workspace_bytes_single(4, 1, 7, 1 << 24, None) > 0
    lc = Launch()
    assert L.twofold_default_launch(0, 4, 1, 7, 1 << 24, 0, ctypes.byref(lc)) == 0
    assert L.twofold_default_launch(0, 8, 1, 7, 1 << 24, 0, ctypes.byref(lc)) == EINVAL
    # the mixed entry points check like the others, before any HIP call
    assert L.twofold_sum_mixed_f32(None, 10, None, fake, ws, big, None) == EINVAL
    assert L.twofold_dot_mixed_f32(fake, None, 10, None, fake, ws, big, None) == EINVAL
    assert L.twofold_sum_mixed_f32(ctypes.c_void_p(0x10002), 10, None, fake, ws, big,
                                   None) == EALIGN
    assert L.twofold_dot_mixed_f32(fake, fake, 10, None, ctypes.c_void_p(0x10004), ws, big,
                                   None) == EALIGN  # binary64 output pair
    assert L.twofold_sum_mixed_f32(fake, 1 << 24, None, fake, ws, 256, None) == EWORKSPACE


def test_binding_checks_caller_outputs():
    """A caller's out tensor must hold the library's rows in the result type:
    a binary32 tensor given for binary64 rows, or too few elements, is
    refused before anything reaches the library (it would be overrun)."""
    import torch
    import paper_1401_0248_amd as tf
    ok = torch.empty((3, 2), dtype=torch.float64)
    assert tf._out(ok, 3, torch.float64, "cpu", (3, 2)) is ok
    assert tf._out(None, 3, torch.float64, "cpu", (3, 2)).shape == (3, 2)
    for bad in (torch.empty((3, 2), dtype=torch.float32), torch.empty((2, 2), dtype=torch.float64),
                torch.empty((3, 4), dtype=torch.float64)[:, :2]):
        with pytest.raises(ValueError):
            tf._out(bad, 3, torch.float64, "cpu", (3, 2))


def test_bench_input_placement():
    """bench.py's input buffer: every array keeps its values, starts 256
    bytes aligned relative to the buffer, and is followed by the gap."""
    import torch
    import bench
    host = {("a", 1): (np.arange(10, dtype=np.float32), np.ones(10, dtype=np.float32)),
            ("b", 2): (np.arange(7, dtype=np.float64), -np.ones(7))}
    d = bench.place_inputs(torch, host, "cpu")
    base = d[("a", 1)][0].data_ptr()
    prev_end = None
    for k, (x, y) in host.items():
        for a, t in zip((x, y), d[k]):
            assert np.array_equal(t.numpy(), a)
            assert (t.data_ptr() - base) % 256 == 0
            if prev_end is not None:
                assert t.data_ptr() - prev_end >= bench.INPUT_GAP
            prev_end = t.data_ptr() + a.nbytes


def test_batch_argument_checks():
    """twofold_batch checks every item on the host before any HIP call."""
    from paper_1401_0248_amd._lib import BatchItem
    L = _lib.load()
    ws = ctypes.c_void_p(0x100000)

    def items(*specs):
        arr = (BatchItem * len(specs))()
        for v, (x, y, out, n, dt, dot, mode) in enumerate(specs):
            arr[v].x, arr[v].y, arr[v].out, arr[v].n = x, y, out, n
            arr[v].dtype, arr[v].is_dot, arr[v].mode = dt, dot, mode
        return arr

    ok = (0x10000, 0x20000, 0x30000, 100, 8, 1, 2)
    big = 1 << 20
    assert L.twofold_batch(items(ok), 65, None, ws, big, None) == EINVAL
    assert L.twofold_batch(items(ok), -1, None, ws, big, None) == EINVAL
    assert L.twofold_batch(None, 2, None, ws, big, None) == EINVAL
    assert L.twofold_batch(None, 0, None, ws, big, None) == 0  # nothing to do
    for bad in ((0x10000, 0x20000, 0x30000, 100, 8, 1, 7),   # mixed: binary32 data only
                (0x10000, 0, 0x30000, 100, 8, 0, 5),         # rounded-product sum
                (0x10000, 0x20000, 0x30000, 100, 2, 1, 2),   # dtype
                (0x10000, 0x20000, 0x30000, -1, 8, 1, 2),    # length
                (0x10000, 0x20000, 0x30000, 100, 8, 2, 2),   # is_dot
                (0x10000, 0x20000, None, 100, 8, 1, 2),      # out
                (None, 0x20000, 0x30000, 100, 8, 1, 2),      # x
                (0x10000, None, 0x30000, 100, 8, 1, 2)):     # y of a dot
        assert L.twofold_batch(items(ok, bad), 2, None, ws, big, None) == EINVAL, bad
    for mis in ((0x10004, 0x20000, 0x30000, 100, 8, 1, 2), (0x10000, 0x20000, 0x30004, 100, 8, 1, 2),
                (0x10000, 0x20000, 0x30004, 100, 4, 1, 7)):  # mixed: binary64 output pair
        assert L.twofold_batch(items(ok, mis), 2, None, ws, big, None) == EALIGN, mis
    # workspace: count times the single-vector one of the largest item's launch
    two = items((0x10000, 0x20000, 0x30000, 1 << 24, 8, 1, 2), (0x10000, 0, 0x30000, 5, 4, 0, 1))
    need = L.twofold_workspace_bytes_batch(two, 2, None)
    one = L.twofold_workspace_bytes_single(8, 1, 2, 1 << 24, None)
    assert need >= 2 * (one - 255)
    assert L.twofold_batch(two, 2, None, ws, need - 256, None) == EWORKSPACE
    assert L.twofold_workspace_bytes_batch(items((0x10000, 0x20000, 0x30000, 100, 8, 1, 7)), 1,
                                           None) == 0
    assert L.twofold_workspace_bytes_batch(items((0x10000, 0x20000, 0x30000, 100, 4, 1, 3)), 1,
                                           None) > 0  # binary64 accumulator of binary32 data


def test_status_codes_of_the_capture_and_tuning_paths():
    from paper_1401_0248_amd._lib import ECAPTURE, ENOTUNED
    L = _lib.load()
    assert (ENOTUNED, ECAPTURE) == (-6, -7)
    for code in (ENOTUNED, ECAPTURE):
        msg = L.twofold_strerror(code)
        assert msg and msg != L.twofold_strerror(12345), code


def test_tuned_launch_reports_measured_rows():
    """Every form the library has was timed by the autotuner for both call
    kinds: twofold_tuned_launch returns OK and the default launch itself."""
    import paper_1401_0248_amd as tf
    L = _lib.load()
    for kind in (0, 1):
        for dt in (4, 8):
            for dot in (0, 1):
                for mode in range(8):
                    if (mode in (5, 6) and not dot) or (mode == 7 and dt == 8):
                        lc = Launch()
                        assert L.twofold_tuned_launch(kind, dt, dot, mode, 100, 3,
                                                      ctypes.byref(lc)) == EINVAL
                        continue
                    for n in (1, 1 << 20, 1 << 31):
                        got, measured = tf.tuned_launch(kind, dt, dot, mode, n, 10)
                        assert measured, (kind, dt, dot, mode, n)
                        want = tf.default_launch(kind, dt, dot, mode, n, 10)
                        assert got.as_dict() == want.as_dict()
    assert L.twofold_tuned_launch(0, 4, 0, 0, 10, 0, None) == EINVAL


def _seg_rows():
    """Segmented rows of the launch table, parsed from its source:
    (dtype, is_dot, mode, n_max, len_max) -> (block, unroll, grid, tile)."""
    import re
    path = os.path.join(os.path.dirname(_lib.__file__), "csrc", "tuned_table.inc")
    big = 2 ** 63 - 1
    rows = []
    for line in open(path):
        m = re.match(r"\{1, (\d+), (\d+), (\d+), (\w+), (\w+), (\d+), (\d+), (\d+), (\d+)\}", line)
        if m:
            v = [big if g == "INT64_MAX" else int(g) for g in m.groups()]
            rows.append((tuple(v[:5]), tuple(v[5:])))
    return rows


def test_short_segments_take_their_own_rows():
    """Every segmented form has a row for short segments (mean length at
    most 1024 elements, any total size), searched first: a batch of short
    segments gets it, one with longer segments the size rows."""
    import paper_1401_0248_amd as tf
    rows = _seg_rows()
    for dt in (4, 8):
        for dot in (0, 1):
            for mode in range(8):
                if (mode in (5, 6) and not dot) or (mode == 7 and dt == 8):
                    continue
                mine = [r for r in rows if r[0][:3] == (dt, dot, mode)]
                short = [r for r in mine if r[0][4] == 1024]
                assert len(short) == 1 and mine[0] == short[0], (dt, dot, mode)
                want = short[0][1]
                n = 1 << 27
                for nseg in (n // 16, n // 1024):  # mean 16 and 1024 elements
                    lc, measured = tf.tuned_launch(1, dt, dot, mode, n, nseg)
                    assert measured
                    assert (lc.block_threads, lc.unroll, lc.grid_blocks, lc.tile_elems) == want
                lc = tf.default_launch(1, dt, dot, mode, n, n // 1025)  # mean 1025
                size_rows = [r for r in mine if r[0][4] != 1024 and n <= r[0][3]]
                assert (lc.block_threads, lc.unroll, lc.grid_blocks, lc.tile_elems) == size_rows[0][1]


def test_batch_item_reserved_must_be_zero():
    from paper_1401_0248_amd._lib import BatchItem
    L = _lib.load()
    arr = (BatchItem * 1)()
    arr[0].x, arr[0].y, arr[0].out, arr[0].n = 0x10000, 0x20000, 0x30000, 100
    arr[0].dtype, arr[0].is_dot, arr[0].mode, arr[0].reserved = 8, 1, 2, 1
    assert L.twofold_batch(arr, 1, None, ctypes.c_void_p(0x100000), 1 << 20, None) == EINVAL
    assert L.twofold_workspace_bytes_batch(arr, 1, None) == 0


SEG_GRID_PROBE = r"""
#include <stdio.h>
#include "kernels.hpp"
int main() {
  const long long ns[] = {0, 1, 3, 4, 5, 20000, 32767, 32768, 32769, 1LL << 26, 1LL << 34,
                          1LL << 56};
  for (long long n : ns) printf("%lld %lld\n", n, (long long)twofold::seg_pass2_blocks(n));
  return 0;
}
"""


def test_segment_combine_grid_is_capped_and_covers_every_segment(tmp_path):
    """The per-segment combine kernel's grid (host arithmetic only): at most
    8192 blocks of four waves for any segment count, and the waves' stride
    loop (wave w takes segments w, w + 4*blocks, ...) reaches every segment
    exactly once."""
    src = tmp_path / "grid.hip"
    src.write_text(SEG_GRID_PROBE)
    exe = tmp_path / "grid"
    r = subprocess.run(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-std=c++17",
                        "-I", os.path.join(ROOT, "paper_1401_0248_amd", "csrc"),
                        "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout
    for line in out.split("\n"):
        if not line:
            continue
        nseg, blocks = (int(v) for v in line.split())
        assert 1 <= blocks <= 8192
        assert blocks * 256 < 2 ** 32  # the x dimension of a launch
        nw = blocks * 4
        assert nw >= min(nseg, 8192 * 4)
        if nseg <= 1 << 20:  # every segment once: waves w < nw take w, w + nw, ...
            seen = np.zeros(nseg, dtype=np.int64)
            for w in range(min(nw, nseg)):
                seen[w::nw] += 1
            assert (seen == 1).all()


def test_launches_report_their_own_status():
    """Every kernel launch of the library goes through launch_kernel, whose
    status is the launch's own (hipLaunchKernel's result): no launch path
    reads the thread's HIP error state, so an error left there by unrelated
    code cannot fail a call between its kernels."""
    csrc = os.path.join(ROOT, "paper_1401_0248_amd", "csrc")
    for f in os.listdir(csrc):
        if f.endswith((".hip", ".hpp")):
            src = open(os.path.join(csrc, f)).read()
            assert "<<<" not in src, f
            if f == "segmented.hip":
                # only plan creation's capture check touches the error state
                # (to clear the errors of its own query and refused
                # allocation), after its last launch-free host work
                body = src[src.index("bool capture_under_way("):src.index("}  // namespace\n\n"
                                                                          "// A plan owns")]
                rest = src.replace(body, "")
                assert "hipGetLastError" not in rest and "hipPeekAtLastError" not in \
                    rest.replace("const bool state_was_clean = hipPeekAtLastError()", ""), f
            else:
                assert "hipGetLastError" not in src, f
                assert "hipPeekAtLastError" not in src, f
