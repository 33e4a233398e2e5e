"""Error paths of the C interface on the GPU, forced from the host so that
every kernel still runs normally:

* an error left in the thread's HIP error state by an unrelated call does
  not change a call's status or result (every launch reports its own
  status);
* plan creation, which allocates and copies synchronously, refuses to run
  while a stream capture is under way (TWOFOLD_ECAPTURE) and leaves the
  capture and the process usable.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_1401_0248_amd as tf
from paper_1401_0248_amd import _lib
from gpu_helpers import DEV, same_bits

pytestmark = pytest.mark.gpu

HIP = ctypes.CDLL("libamdhip64.so")
HIP.hipSetDevice.argtypes = [ctypes.c_int]
HIP.hipGetDeviceCount.argtypes = [ctypes.POINTER(ctypes.c_int)]
HIP.hipStreamCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
HIP.hipStreamBeginCapture.argtypes = [ctypes.c_void_p, ctypes.c_int]
HIP.hipStreamEndCapture.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
HIP.hipGraphDestroy.argtypes = [ctypes.c_void_p]
HIP.hipStreamDestroy.argtypes = [ctypes.c_void_p]
HIP.hipPeekAtLastError.argtypes = []
HIP.hipGetLastError.argtypes = []

HIP_STREAM_DEFAULT, HIP_STREAM_NON_BLOCKING = 0, 1
CAPTURE_GLOBAL = 0  # hipStreamCaptureModeGlobal


def _plant_stale_error():
    """Leave an error in this thread's HIP error state with a harmless call:
    selecting a device that does not exist (the current device stays)."""
    n = ctypes.c_int(0)
    assert HIP.hipGetDeviceCount(ctypes.byref(n)) == 0
    assert HIP.hipSetDevice(n.value + 7) != 0
    assert HIP.hipPeekAtLastError() != 0


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_stale_error_does_not_fail_a_call(dtype):
    x = torch.linspace(-1, 1, 1 << 20, dtype=dtype, device=DEV) * 0.3
    y = torch.linspace(1, -2, 1 << 20, dtype=dtype, device=DEV)
    lc = tf.Launch(256, 4, 64, 0, 0)  # two kernels: blocks, then the combine
    off = torch.tensor([0, 5, 70000, 1 << 20], dtype=torch.int64, device=DEV)
    ref = tf.dot(x, y, "rigorous", lc)
    ref_seg = tf.segdot(x, y, off)
    outs = {"dot": torch.empty(2, dtype=dtype, device=DEV),
            "segdot": torch.empty((3, 2), dtype=dtype, device=DEV),
            "batch": torch.empty(2, dtype=dtype, device=DEV)}
    tf.batch([(x, y, "rigorous")], lc, outs=[outs["batch"]])  # caches the workspace
    torch.cuda.synchronize()
    for call in ("dot", "segdot", "batch"):
        # the error is planted after all torch work of the step, right before
        # the library call, and cleared right after it (torch's own launch
        # checks read the thread's error state)
        _plant_stale_error()
        try:
            if call == "dot":
                got = tf.dot(x, y, "rigorous", lc, out=outs[call])  # raises on nonzero status
                want = ref
            elif call == "segdot":
                got = tf.segdot(x, y, off, out=outs[call])
                want = ref_seg
            else:
                got = tf.batch([(x, y, "rigorous")], lc, outs=[outs[call]])[0]
                want = ref
        finally:
            HIP.hipGetLastError()
        torch.cuda.synchronize()
        a = got.double().cpu().numpy().ravel()
        b = want.double().cpu().numpy().ravel()
        assert same_bits(a, b), call


def _plan_create(offsets):
    L = _lib.load()
    h = np.ascontiguousarray(offsets, dtype=np.int64)
    plan = ctypes.c_void_p()
    rc = L.twofold_seg_plan_create(h.ctypes.data, h.size - 1, 8, 1, 2, None, ctypes.byref(plan))
    return rc, plan


@pytest.mark.parametrize("flags", [HIP_STREAM_DEFAULT, HIP_STREAM_NON_BLOCKING],
                         ids=["blocking-stream", "non-blocking-stream"])
def test_plan_create_during_capture_is_refused(flags):
    """A global-mode capture on a stream of its own (no work recorded):
    plan creation returns TWOFOLD_ECAPTURE and allocates nothing; the capture
    is then ended and the same creation succeeds outside it."""
    torch.cuda.synchronize()
    HIP.hipGetLastError()  # start from a clean error state
    st = ctypes.c_void_p()
    assert HIP.hipStreamCreateWithFlags(ctypes.byref(st), flags) == 0
    graph = ctypes.c_void_p()
    try:
        assert HIP.hipStreamBeginCapture(st, CAPTURE_GLOBAL) == 0
        rc, plan = _plan_create([0, 10, 20, 4096])
        # the refusal leaves no error behind for the caller's next check
        left = HIP.hipPeekAtLastError()
        end = HIP.hipStreamEndCapture(st, ctypes.byref(graph))
        HIP.hipGetLastError()  # whatever ending the capture reported is the test's own
        if rc == _lib.OK:  # not refused: release what was made before failing
            _lib.load().twofold_seg_plan_destroy(plan)
        assert rc == _lib.ECAPTURE, (rc, end)
        assert not plan.value
        assert left == 0, left
    finally:
        if graph.value:
            HIP.hipGraphDestroy(graph)
        HIP.hipStreamDestroy(st)
    # outside the capture the same plan builds and runs
    rc, plan = _plan_create([0, 10, 20, 4096])
    assert rc == _lib.OK
    assert _lib.load().twofold_seg_plan_destroy(plan) == 0
    x = torch.ones(4096, dtype=torch.float64, device=DEV)
    p = tf.SegPlan(np.array([0, 10, 20, 4096]), torch.float64, True, "rigorous")
    out = p.execute(x, x)
    torch.cuda.synchronize()
    assert out[:, 0].cpu().tolist() == [10.0, 10.0, 4076.0]
    p.close()
