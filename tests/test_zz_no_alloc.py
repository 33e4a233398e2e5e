"""The allocation-free batch entry point (twofold_batch_static), through the
C interface: its pairs equal twofold_batch's bit for bit with the same
items and launch, on two calls in a row (the second with smaller inputs, so
the static scratch holds the first call's pairs when it starts), and a batch
that needs more than the scratch is refused before any HIP call."""
import ctypes

import numpy as np
import pytest
import torch

from paper_1401_0248_amd import _lib
from paper_1401_0248_amd._lib import EWORKSPACE, BatchItem, Launch

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SCRATCH = 4 << 20


def _items(specs):
    """specs: (x, y, out, mode) tensors; returns the C item array."""
    arr = (BatchItem * len(specs))()
    for v, (x, y, out, mode) in enumerate(specs):
        arr[v].x = x.data_ptr()
        arr[v].y = y.data_ptr() if y is not None else None
        arr[v].out = out.data_ptr()
        arr[v].n = x.numel()
        arr[v].dtype = x.element_size()
        arr[v].is_dot = int(y is not None)
        arr[v].mode = mode
    return arr


def _data(n, seed):
    g = torch.Generator(device="cpu").manual_seed(seed)
    x64 = (torch.rand(n, generator=g, dtype=torch.float64) * 2 - 1).to(DEV)
    y64 = (torch.rand(n, generator=g, dtype=torch.float64) * 2 - 1).to(DEV)
    # a binary32 pair at an odd element offset (head and tail peeled)
    x32 = (torch.rand(n + 3, generator=g, dtype=torch.float64) * 2 - 1).float().to(DEV)[3:]
    y32 = (torch.rand(n + 3, generator=g, dtype=torch.float64) * 2 - 1).float().to(DEV)[3:]
    return x64, y64, x32, y32


def _run(L, n, seed, lc):
    x64, y64, x32, y32 = _data(n, seed)
    # (x, y, mode, output dtype): rigorous and fast dots, a Kahan sum, the
    # wider accumulator and the mixed form (binary64 results)
    forms = [(x64, y64, 2, torch.float64), (x32, y32, 1, torch.float32), (x64, None, 4, torch.float64),
             (x32, y32, 3, torch.float64), (x32, None, 7, torch.float64)]
    outs_ref = [torch.full((2,), float("nan"), dtype=d, device=DEV) for *_, d in forms]
    outs_static = [torch.full((2,), float("nan"), dtype=d, device=DEV) for *_, d in forms]
    ref = _items([(x, y, o, m) for (x, y, m, _), o in zip(forms, outs_ref)])
    sta = _items([(x, y, o, m) for (x, y, m, _), o in zip(forms, outs_static)])
    count = len(forms)
    lp = ctypes.byref(lc) if lc is not None else None
    need = L.twofold_workspace_bytes_batch(ctypes.cast(ref, ctypes.c_void_p), count, lp)
    ws = torch.empty(need + 256, dtype=torch.uint8, device=DEV)
    wp = (ws.data_ptr() + 255) & ~255
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.twofold_batch(ctypes.cast(ref, ctypes.c_void_p), count, lp, ctypes.c_void_p(wp), need,
                           st) == 0
    assert L.twofold_batch_static(ctypes.cast(sta, ctypes.c_void_p), count, lp, st) == 0
    torch.cuda.synchronize()
    for a, b in zip(outs_ref, outs_static):
        assert torch.equal(a.view(torch.int8), b.view(torch.int8)), (a, b)
        assert torch.isfinite(a).all()


@pytest.mark.parametrize("lc", [None, Launch(256, 4, 512, 0, 0), Launch(1024, 8, 7, 0, 0)],
                         ids=["default", "256x4x512", "1024x8x7"])
def test_static_batch_equals_batch_twice(lc):
    L = _lib.load()
    _run(L, (1 << 22) + 5, 1, lc)  # larger first: fills more of the scratch
    _run(L, 70001, 2, lc)          # then smaller, on top of what the first left


def test_static_batch_refuses_oversized_pairs():
    L = _lib.load()
    x = torch.zeros(1 << 16, dtype=torch.float64, device=DEV)
    out = torch.zeros(2 * 64, dtype=torch.float64, device=DEV)
    specs = [(x, x, out[2 * v:2 * v + 2], 2) for v in range(64)]
    arr = _items(specs)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    # 64 items x 8192 blocks x 16 bytes = 8 MiB of block pairs > 4 MiB
    big = Launch(256, 1, 8192, 0, 0)
    assert 64 * 8192 * 16 > SCRATCH
    assert L.twofold_batch_static(ctypes.cast(arr, ctypes.c_void_p), 64, ctypes.byref(big), st) \
        == EWORKSPACE
    # exactly at the limit: 64 items x 4096 blocks x 16 bytes = 4 MiB
    edge = Launch(256, 1, 4096, 0, 0)
    assert L.twofold_batch_static(ctypes.cast(arr, ctypes.c_void_p), 64, ctypes.byref(edge), st) == 0
    torch.cuda.synchronize()
    assert (out[0::2] == 0).all()
