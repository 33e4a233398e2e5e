"""GPU parity of the precision monitor (twofold_monitor) against the
oracle's flags (oracle/monitor.py), on seeded synthetic pairs and on the
order model's pairs of a segmented batch. Flags and counts must match
exactly."""
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_1401_0248_amd as tf
import synth
from gpu_helpers import DEV
from oracle import monitor

pytestmark = pytest.mark.gpu

TDT = {np.float32: torch.float32, np.float64: torch.float64}


def _note(msg):
    print("[monitor] " + msg, file=sys.stderr, flush=True)


def _pairs(dtype, count, seed, tau):
    """Seeded (value, error) rows mixing ordinary pairs, zeros, subnormals,
    non-finite values and pairs exactly at and just above the threshold."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal(count) * np.exp2(rng.integers(-40, 40, count))
    e = v * np.exp2(rng.integers(-40, 2, count).astype(np.float64)) * rng.choice([-1, 1], count)
    kind = rng.integers(0, 10, count)
    tiny = np.finfo(dtype).smallest_subnormal
    v = np.where(kind == 0, 0.0, v)
    e = np.where(kind == 1, 0.0, e)
    e = np.where(kind == 2, tiny * rng.integers(1, 4, count), e)
    v = np.where(kind == 3, np.inf, v)
    e = np.where(kind == 4, np.nan, e)
    pairs = np.stack([v, e], axis=1).astype(dtype)
    # exact-threshold rows: e = tau * |v| when that product is exact in dtype
    k = np.flatnonzero(kind == 5)
    pv = pairs[k, 0].astype(np.float64)
    pairs[k, 1] = (tau * np.abs(pv)).astype(dtype)
    k2 = np.flatnonzero(kind == 6)
    pairs[k2, 1] = np.nextafter((tau * np.abs(pairs[k2, 0].astype(np.float64))).astype(dtype),
                                dtype(np.inf))
    return np.ascontiguousarray(pairs)


def _lengths(dtype, count, seed):
    rng = np.random.default_rng(seed + 1)
    inv_u = monitor.inv_unit_roundoff(dtype)
    lens = rng.integers(0, 1 << 20, count).astype(np.int64)
    if count:
        special = np.array([inv_u - 1, inv_u, inv_u + 1, 0], dtype=np.int64)
        pick = rng.integers(0, count, special.size * 3)
        lens[pick] = np.tile(special, 3)
    return lens


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("count", [0, 1, 63, 1000, 1_000_003])
def test_flags_match_oracle(dtype, count):
    tau = 2.0 ** -20
    _note("%s count %d" % (np.dtype(dtype).name, count))
    pairs = _pairs(dtype, count, 3 + count, tau)
    lens = _lengths(dtype, count, 5 + count)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pd = torch.from_numpy(pairs).to(DEV)
    od = torch.from_numpy(off).to(DEV)
    flags, nf = tf.monitor(pd, tau, offsets=od)
    want = np.array(monitor.flags(pairs, lens, tau, dtype), dtype=np.int64)
    got = flags.cpu().numpy().astype(np.int64)
    assert np.array_equal(got, want)
    assert int(nf.item()) == int(np.count_nonzero(want))
    # one length for all
    for n in (5, monitor.inv_unit_roundoff(dtype)):
        flags, nf = tf.monitor(pd, tau, n=n)
        want = np.array(monitor.flags(pairs, [n] * count, tau, dtype), dtype=np.int64)
        assert np.array_equal(flags.cpu().numpy().astype(np.int64), want)
        assert int(nf.item()) == int(np.count_nonzero(want))


def test_monitor_of_a_segmented_batch():
    """Binary32 rigorous dots of ill-conditioned segments: the GPU pairs
    equal the order model's (checked first), and the monitor's flags equal
    the oracle's flags of the model's pairs."""
    lengths = synth.segment_lengths(11, 400, max_len=1 << 14)
    off = synth.offsets_from_lengths(lengths)
    n = int(off[-1])
    x, y = synth.illcond_dot(synth.illcond_seed(12), n + n % 2, 1e12, np.float32)
    x, y = np.ascontiguousarray(x[:n]), np.ascontiguousarray(y[:n])
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.from_numpy(y).to(DEV)
    od = torch.from_numpy(np.asarray(off, dtype=np.int64)).to(DEV)
    lc = tf.Launch(256, 4, 64, 0, 4096)
    out = tf.segdot(xd, yd, od, "rigorous", lc)
    mis = (xd.data_ptr() % 16) // 4
    model = oracle.model_seg("rigorous", x, off, y, mis, 4, 4096)
    got = out.double().cpu().numpy()
    assert np.array_equal(got.view(np.uint64), model.view(np.uint64))
    for tau in (0.0, 2.0 ** -30, 2.0 ** -24, 1e-3):
        flags, nf = tf.monitor(out, tau, offsets=od)
        want = np.array(monitor.flags(model.astype(np.float32), np.diff(off), tau, np.float32))
        assert np.array_equal(flags.cpu().numpy().astype(np.int64), want.astype(np.int64)), tau
        assert int(nf.item()) == int(np.count_nonzero(want))


def test_monitor_in_a_graph():
    """Plan execute and monitor captured together; every replay (with eager
    work in between) gives the eager flags and count."""
    lengths = synth.segment_lengths(13, 300, max_len=1 << 14)
    off = synth.offsets_from_lengths(lengths)
    x, y = synth.uniform(14, int(off[-1]), np.float64, count=2)
    xd = torch.from_numpy(x).to(DEV)
    yd = torch.from_numpy(y).to(DEV)
    od = torch.from_numpy(np.asarray(off, dtype=np.int64)).to(DEV)
    plan = tf.SegPlan(off, torch.float64, True, "fast")
    tau = 2.0 ** -50
    out = plan.execute(xd, yd)
    f0, n0 = tf.monitor(out, tau, offsets=od)
    f0, n0 = f0.clone(), n0.clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        ws = tf.workspace(plan.workspace_bytes, xd.device)
    flags = torch.empty_like(f0)
    nf = torch.empty_like(n0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.execute(xd, yd, out=out, ws=ws)
        tf.monitor(out, tau, offsets=od, flags=flags, nflagged=nf)
    for i in range(5):
        flags.fill_(-1)
        nf.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(flags, f0) and torch.equal(nf, n0), i
        tf.monitor(out, 0.5, offsets=od)  # eager work between replays
        torch.cuda.synchronize()
