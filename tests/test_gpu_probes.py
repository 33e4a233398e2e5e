"""The instruments on the GPU: the read probe must fold every byte it was
given (the OR of all its 32-bit words equals the OR over the arrays, for
aligned and ragged lengths and every launch shape), and the compute probe
must be deterministic for every form."""
import numpy as np
import pytest
import torch

import paper_1401_0248_amd as tf
from gpu_helpers import DEV

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("two", [False, True])
def test_read_probe_reads_every_word(two):
    rng = np.random.default_rng(9)
    for nvec in (1, 7, 4096, 65536 + 5, 1 << 20):
        for bt, u, gb in ((64, 1, 1), (256, 4, 7), (512, 8, 33), (1024, 2, 300)):
            # one set bit per word position, somewhere: only a full read sees all
            x = np.zeros(nvec * 4, dtype=np.uint32)
            y = np.zeros(nvec * 4, dtype=np.uint32)
            for b in range(32):
                x[rng.integers(0, x.size)] |= np.uint32(1 << b)
            if two:
                y[x.size - 1] = np.uint32(0x80000001)
            xd = torch.from_numpy(x.view(np.int32)).to(DEV)
            yd = torch.from_numpy(y.view(np.int32)).to(DEV) if two else None
            sink = tf.probe_read(xd, yd, tf.Launch(bt, u, gb, 0, 0)).cpu().numpy()
            got = int(np.bitwise_or.reduce(sink.astype(np.uint64)))
            want = int(np.bitwise_or.reduce(x)) | (int(np.bitwise_or.reduce(y)) if two else 0)
            assert got == want, (nvec, bt, u, gb)
            assert want == 0xFFFFFFFF


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_compute_probe_deterministic(dtype):
    seed = torch.linspace(-1, 1, 64, dtype=dtype, device=DEV)
    lc = tf.Launch(128, 4, 5, 0, 0)
    for is_dot in (False, True):
        forms = ["plain", "fast", "rigorous", "kahan", "wide"]
        if is_dot:
            forms += ["fast_rounded", "rigorous_rounded"]
        if dtype == torch.float32:
            forms += ["mixed"]
        for form in forms:
            a = tf.probe_compute(seed, is_dot, form, 100, lc).cpu().numpy()
            b = tf.probe_compute(seed, is_dot, form, 100, lc).cpu().numpy()
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), (is_dot, form)
            assert np.all(np.isfinite(a)), (is_dot, form)
            assert np.any(a != 0), (is_dot, form)
