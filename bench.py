"""Benchmark: twofold dot products of ill-conditioned vectors on one GPU.

Workload (one step): the fast and the rigorous twofold dot of 12 resident
vector pairs of N = 2^24 elements, binary32 and binary64, generated with
target conditions 1e6, 1e8, ..., 1e16 (synth.illcond_dot). The step is one
mixed batch call: the 24 dots in one launch and one combine kernel; the
rigorous dots run first, so no pair is re-read while it could still sit in
the 256 MB last-level cache. Prints one JSON line.

The dominant kernel is the batch (4.5 GiB per launch); its average duration
is measured with a pair of HIP events on the launch stream around the timed
steps (a step is that launch alone) and gives the roofline entry (algorithmic bytes / time vs 8 TB/s). Every dot is
checked bit for bit against its single-vector call with the same launch
after the timed region, and the binary64 rigorous single calls are timed for
reference. The CPU-baseline leg, the only part that runs the oracle, times
the oracle's sequential paper-order loops on one host thread over the same
inputs and grades every form's GPU result against the exact sum.
"""
import argparse
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "twofold dot/sum Gelem/s & %HBM peak; FP32-twofold vs FP64-plain at equal err"
HBM_PEAK_GBS = 8000.0
N = 1 << 24
DECADES = (6, 8, 10, 12, 14, 16)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def make_inputs():
    import numpy as np
    import synth

    jobs = [(dt, d) for dt in (np.float32, np.float64) for d in DECADES]

    def one(job):
        dt, d = job
        return job, synth.illcond_dot(synth.illcond_seed(d), N, 10.0 ** d, dt)

    with ThreadPoolExecutor(max_workers=min(12, os.cpu_count() or 4)) as ex:
        return dict(ex.map(one, jobs))


# Gap after every input array in the device buffer. x and y of a dot are
# read at the same index at the same time, and their placement moves the
# rate: with the arrays adjacent (x and y exactly 128 MiB apart for 2^24
# binary64 elements) the step measured about 3% slower than with a 4 KiB gap
# after every array. The gap keeps every array 256-byte aligned.
INPUT_GAP = 4096


def place_inputs(torch, host, dev):
    """The 12 pairs in one device buffer, each array followed by the gap;
    returns {key: (x, y)} device views."""
    def slot(a):
        return (a.nbytes + 255) // 256 * 256 + INPUT_GAP

    total = sum(slot(x) + slot(y) for x, y in host.values())
    buf = torch.empty(total, dtype=torch.uint8, device=dev)
    out, off = {}, 0
    for k, (x, y) in host.items():
        views = []
        for a in (x, y):
            t = buf[off:off + a.nbytes].view(torch.from_numpy(a[:1]).dtype)
            t.copy_(torch.from_numpy(a))
            views.append(t)
            off += slot(a)
        out[k] = tuple(views)
    return out


def gpu_results(dev_in, tf):
    """Every form's pair for every input (outside the timed region)."""
    import numpy as np

    res = {}
    for k, (xd, yd) in dev_in.items():
        for mode in ("plain", "fast", "rigorous"):
            res[k + (mode,)] = tf.dot(xd, yd, mode).double().cpu().numpy()
        res[k + ("dotd",)] = tf.dotd(xd, yd).cpu().numpy()
        if k[0] == np.float32:
            res[k + ("mixed",)] = tf.dot_mixed(xd, yd).cpu().numpy()
    return res


def host_info():
    """CPU model string and the cores this process may run on."""
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return {"cpu": model, "cores_available": avail}


def exact_timing(oracle, x, y):
    """Gelem/s of the oracle's exact accumulator on one pair, on one thread
    and on every thread it uses by default."""
    res = {}
    for label, nt in (("1_thread", 1), ("all_threads", oracle.default_threads())):
        t0 = time.perf_counter()
        oracle.Exact(x, y, nthreads=nt)
        res[label] = {"threads": nt, "gelem_s": round(x.size / (time.perf_counter() - t0) / 1e9, 4)}
    return res


def oracle_leg(host, gpu, launches, perm_host=None, perm_gpu=None):
    """The CPU-baseline leg, the only part of the benchmark that runs the
    oracle: (1) times the oracle's sequential rigorous and fast twofold dots
    (paper order, FMA remainder) over every input of one step on one host
    thread, and its exact accumulator on one pair; (2) grades the GPU's pairs
    against the exact accumulator: |v + e - S| / sum|x y| and |v - S| /
    sum|x y|, median over the conditions, the estimate quality
    q = e / (S - v), and for the rigorous form the largest ratio of the
    error to the proven bound of the launch's own tree."""
    import numpy as np

    import oracle
    from oracle import bounds

    t0 = time.perf_counter()
    elems = 0
    for (dt, d), (x, y) in host.items():
        oracle.seq("dott", x, y)
        oracle.seq("dottf", x, y)
        elems += 2 * x.size
    dt_s = time.perf_counter() - t0
    base = {"value": round(elems / dt_s / 1e9, 4), "unit": "Gelem/s", "cores": 1, "kind": "oracle",
            "sample": "one full step: sequential rigorous + fast twofold dot (paper order, FMA "
                      "remainder) over the 12 ill-conditioned pairs, N=2^24 each, %.1f s" % dt_s,
            "host": host_info(),
            "exact_accumulator": dict(sample="binary64 pair of target cond 1e16, N=2^24",
                                      **exact_timing(oracle, *host[(np.float64, 16)]))}
    rows = {}
    for (dt, d), (x, y) in host.items():
        ex = oracle.Exact(x, y)
        key = "f32" if dt == np.float32 else "f64"
        for mode in ("plain", "fast", "rigorous"):
            p = gpu[(dt, d, mode)]
            rows.setdefault("%s_%s" % (key, mode), []).append(abs(ex.diff(p[0], p[1])) / ex.A)
            if mode == "rigorous":
                lc = launches[(dt, mode)]
                tb = bounds.single_bound(dt, x.size, lc.block_threads, lc.unroll, lc.grid_blocks,
                                         ex.A)
                rows.setdefault("%s_rigorous_over_tree_bound" % key, []).append(
                    abs(ex.diff(p[0], p[1])) / tb)
                u = bounds.unit_roundoff(dt)
                rows.setdefault("%s_rigorous_over_4Nu2_bound" % key, []).append(
                    abs(ex.diff(p[0], p[1])) / (4 * x.size * u * u * ex.A))
            if mode != "plain":
                dv = ex.diff(p[0])  # v - S, rounded once
                rows.setdefault("%s_%s_value" % (key, mode), []).append(abs(dv) / ex.A)
                rows.setdefault("%s_%s_q" % (key, mode), []).append(
                    p[1] / -dv if dv else float("nan"))
        p = gpu[(dt, d, "dotd")]
        if dt == np.float32:
            rows.setdefault("f32data_f64plain", []).append(abs(ex.diff(p[0])) / ex.A)
            p = gpu[(dt, d, "mixed")]
            rows.setdefault("f32_mixed", []).append(abs(ex.diff(p[0], p[1])) / ex.A)
        else:
            rows.setdefault("f64_double_word", []).append(abs(ex.diff(p[0], p[1])) / ex.A)
        rows.setdefault("cond_" + key, []).append(2 * ex.A / abs(ex.S) if ex.S else float("inf"))
    if perm_host:
        pr = {"measure": "|v + e - S| / sum|x y| on the target-cond-1e16 pairs under a seeded "
                         "permutation (running sums no longer cancel in order)"}
        for dt, (x, y) in perm_host.items():
            ex = oracle.Exact(x, y)
            key = "f32" if dt == np.float32 else "f64"
            for mode in ("plain", "fast", "rigorous"):
                p = perm_gpu[(dt, mode)]
                pr["%s_%s" % (key, mode)] = float("%.3g" % (abs(ex.diff(p[0], p[1])) / ex.A))
            p = perm_gpu[(dt, "dotd")]
            pr["f32data_f64plain" if dt == np.float32 else "f64_double_word"] = float(
                "%.3g" % (abs(ex.diff(p[0], p[1])) / ex.A))
            if dt == np.float32:
                p = perm_gpu[(dt, "mixed")]
                pr["f32_mixed"] = float("%.3g" % (abs(ex.diff(p[0], p[1])) / ex.A))
    acc = {"measure": "median over conditions of |v + e - S| / sum|x y| (*_value: |v - S| / "
                      "sum|x y|; *_q: e / (S - v); *_over_tree_bound and *_over_4Nu2_bound: the "
                      "largest |v + e - S| over the proven bound of the launch's reduction "
                      "tree, and over 4 N u^2 sum|x y|)"}
    for k, v in rows.items():
        if k.startswith("cond_"):
            acc[k] = ["%.3g" % c for c in v]
        elif k.endswith("_bound"):
            acc[k] = float("%.3g" % max(v))
        else:
            acc[k] = float("%.3g" % np.median(v))
    if perm_host:
        acc["permuted"] = pr
    return base, acc


def precision_study(torch, tf, dev, with_oracle):
    """The binary32 precision form: N = 2^26 binary32 pairs x = m 2^k, y
    likewise (m uniform(-1, 1), k uniform integer in [-20, 20], seed 2).
    Times the binary32 plain, fast and rigorous twofold dots, the mixed
    form (binary32 rigorous value, binary64 error term), the binary64 plain
    dot of the same binary32 data (dotd) and the binary64 plain and
    rigorous dots over a binary64 copy (twice the bytes), HIP-graph replay.
    Its CPU-baseline leg grades every result against the exact accumulator
    and times the oracle's sequential rigorous dot on the same data. One
    JSON line."""
    import numpy as np
    import synth

    n = 1 << 26
    log("precision study: generating N=2^26 scaled binary32 pairs")
    x, y = synth.scaled(2, n)
    xd, yd = torch.from_numpy(x).to(dev), torch.from_numpy(y).to(dev)
    x64, y64 = xd.double(), yd.double()
    L = tf._lib.load()
    ws = tf.Workspace(max(L.twofold_workspace_bytes_single(sz, 1, m, n, None)
                          for sz, m in ((4, 0), (4, 1), (4, 2), (4, 3), (4, 7), (8, 0), (8, 2),
                                        (8, 3))),
                      dev)
    forms = [("f32 plain", lambda o: tf.dot(xd, yd, "plain", out=o, ws=ws), 4),
             ("f32 fast twofold", lambda o: tf.dot(xd, yd, "fast", out=o, ws=ws), 4),
             ("f32 rigorous twofold", lambda o: tf.dot(xd, yd, "rigorous", out=o, ws=ws), 4),
             ("f32 rigorous twofold, f64 error term (mixed)",
              lambda o: tf.dot_mixed(xd, yd, out=o, ws=ws), 8),
             ("f64 plain on f32 data (dotd)", lambda o: tf.dotd(xd, yd, out=o, ws=ws), 8),
             ("f64 plain on an f64 copy", lambda o: tf.dot(x64, y64, "plain", out=o, ws=ws), 8),
             ("f64 rigorous on an f64 copy", lambda o: tf.dot(x64, y64, "rigorous", out=o, ws=ws),
              8),
             ("f64 double-word (dotd) on an f64 copy", lambda o: tf.dotd(x64, y64, out=o, ws=ws),
              8)]
    rows, results = [], {}
    for name, fn, osz in forms:
        o = torch.empty(2, dtype=torch.float64, device=dev)
        ov = o if osz == 8 else o.view(torch.float32)[:2]
        t, tmin = graph_time(torch, lambda: (fn(ov), 1)[1])
        results[name] = ov.double().cpu().numpy()
        nbytes = 2 * n * (4 if "f32 data" in name or name.startswith("f32") else 8)
        rows.append({"form": name, "us": round(t * 1e6, 2), "us_min": round(tmin * 1e6, 2),
                     "gelem_s": round(n / t / 1e9, 1), "gb_s": round(nbytes / t / 1e9, 1),
                     "hbm_frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4)})
        log("  %-30s %8.2f us %7.1f Gelem/s" % (name, t * 1e6, n / t / 1e9))
    res = {"device": device_info(torch, dev),
           "workload": "precision form: binary32 twofold vs binary64 plain, N=2^26, "
                       "x, y = uniform(-1,1) * 2^k, k in [-20, 20], seed 2",
           "n": n, "rows": rows}
    if with_oracle:
        import oracle
        log("precision study: cpu baseline leg (exact grading, sequential oracle timing)")
        ex = oracle.Exact(x, y)
        for r in rows:
            v, e = results[r["form"]]
            r["err_rel"] = float("%.3g" % (abs(ex.diff(v, e)) / ex.A))
        t0 = time.perf_counter()
        oracle.seq("dott", x, y)
        dt_s = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(n / dt_s / 1e9, 4), "unit": "Gelem/s", "cores": 1,
                               "kind": "oracle", "sample": "sequential rigorous twofold dot "
                               "(paper order, FMA remainder) of the whole pair, %.1f s" % dt_s,
                               "host": host_info()}
        res["err_measure"] = "|v + e - S| / sum|x y| against the exact accumulator"
    print(json.dumps(res), flush=True)


COPY_BYTES = 1 << 28
FORMS = ("plain", "fast", "rigorous")


def device_info(torch, dev):
    """Name, architecture, compute units and memory of the device."""
    p = torch.cuda.get_device_properties(dev)
    return {"name": p.name, "arch": getattr(p, "gcnArchName", ""),
            "compute_units": p.multi_processor_count, "memory_gib": round(p.total_memory / 2 ** 30, 1)}


def graph_time(torch, calls, reps=30):
    """(median, min) seconds per call over `reps` replays of a graph of
    calls()."""
    import statistics
    calls()
    torch.cuda.synchronize()
    cap = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cap):
        ncalls = calls()
    g.replay()
    torch.cuda.synchronize()
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        g.replay()
        e1.record(st)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3 / ncalls)
    return statistics.median(ts), min(ts)


SCRUB_BYTES = 1 << 29


def cold_time(torch, call, scrub, reps=30):
    """Median seconds of one call whose inputs were evicted from every cache
    level: each rep first reads and writes a 512 MiB scrub buffer (longer
    than the host needs to enqueue the call, so the events around the call
    time it back to back on the device)."""
    import statistics
    st = torch.cuda.current_stream()
    ts = []
    for _ in range(reps):
        scrub.add_(1.0)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        call()
        e1.record(st)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3)
    return statistics.median(ts)


def to_device_chunks(torch, chunks, n, dtype, dev):
    t = torch.empty(n, dtype=dtype, device=dev)
    i = 0
    for c in chunks:
        t[i:i + c.size].copy_(torch.from_numpy(c))
        i += c.size
    return t


def roofline_sweep(torch, tf, dev):
    """Every form of sum and dot (plain, fast, rigorous, Kahan, the wide
    accumulator, for binary32 data the mixed form, and for dots the paper's
    rounded-product fast and rigorous forms), binary32 and binary64, at
    N = 4096, 2^20 and
    1 GiB per vector, uniform(-1, 1) data of seed 1, tuned default
    launches, HIP-graph replay: the method comparison of the paper's
    Table 1 on one MI355X. One JSON line."""
    import numpy as np
    import synth

    rows = []
    scrub = torch.zeros(SCRUB_BYTES // 4, dtype=torch.float32, device=dev)
    for dtype, tdt in ((np.float32, torch.float32), (np.float64, torch.float64)):
        size = np.dtype(dtype).itemsize
        for n in (4096, 1 << 20, (1 << 30) // size):
            log("sweep %s n=%d" % (np.dtype(dtype).name, n))
            rng_chunks = synth.uniform_chunks(1, 2 * n, dtype)
            both = to_device_chunks(torch, rng_chunks, 2 * n, tdt, dev)
            x, y = both[:n], both[n:]  # x drawn entirely, then y
            big = n * size >= (1 << 28)
            reps = 4 if big else 50  # calls per graph: amortizes the replay's own start
            for op in ("sum", "dot"):
                forms = FORMS + ("kahan", "wide")
                if op == "dot":
                    forms += ("fast_rounded", "rigorous_rounded")
                if size == 4:
                    forms += ("mixed",)
                for form in forms:
                    out = torch.empty(2, dtype=torch.float64, device=dev)
                    o = out if (size == 8 or form in ("wide", "mixed")) else out.view(torch.float32)[:2]
                    need = tf._lib.load().twofold_workspace_bytes_single(
                        size, op == "dot", tf.mode_id(form), n, None)
                    ws = tf.Workspace(need, dev)

                    def one():
                        if form == "wide":
                            (tf.dotd(x, y, out=o, ws=ws) if op == "dot"
                             else tf.sumd(x, out=o, ws=ws))
                        elif form == "mixed":
                            (tf.dot_mixed(x, y, out=o, ws=ws) if op == "dot"
                             else tf.sum_mixed(x, out=o, ws=ws))
                        elif op == "dot":
                            tf.dot(x, y, form, out=o, ws=ws)
                        else:
                            tf.sum(x, form, out=o, ws=ws)

                    def calls():
                        for _ in range(reps):
                            one()
                        return reps

                    t, tmin = graph_time(torch, calls)
                    first = o.clone()
                    nbytes = n * size * (2 if op == "dot" else 1)
                    row = {"dtype": np.dtype(dtype).name, "op": op, "form": form, "n": n,
                           "us": round(t * 1e6, 3), "us_min": round(tmin * 1e6, 3),
                           "gelem_s": round(n / t / 1e9, 2), "gb_s": round(nbytes / t / 1e9, 1),
                           "hbm_frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4)}
                    if not big:
                        row["us_cold"] = round(cold_time(torch, one, scrub) * 1e6, 3)
                    row["bitwise_repeatable"] = bool(torch.equal(first.view(torch.int8),
                                                                 o.view(torch.int8)))
                    rows.append(row)
                    log("  %s %-16s %10.2f us %8.1f GB/s" % (op, form, t * 1e6, nbytes / t / 1e9))
            del both, x, y
            torch.cuda.empty_cache()
    print(json.dumps({"device": device_info(torch, dev),
                      "workload": "roofline sweep, uniform(-1,1) seed 1, tuned default launches; "
                                  "us = median over 30 graph replays of 50 calls (4 at 1 GiB) "
                                  "per call, warm; us_cold = one call after a 512 MiB scrub",
                      "peak_gb_s": HBM_PEAK_GBS, "rows": rows}), flush=True)


def segmented_batch(torch, tf, dev):
    """20,000 segment pairs with log-uniform lengths in [1, 2^20] (seed 3,
    1,504,333,896 elements), and the secondary variant capped at 2^17
    (221,217,512 elements); uniform(-1, 1) data of seed 3 (x, then y),
    binary32 and binary64, fast and rigorous dots through plans with the
    tuned default launch, HIP-graph replay. One JSON line."""
    import numpy as np
    import synth

    rows = []
    for dtype, tdt in ((np.float32, torch.float32), (np.float64, torch.float64)):
        for cap in (1 << 20, 1 << 17):
            lengths = synth.segment_lengths(3, 20000, max_len=cap)
            off = synth.offsets_from_lengths(lengths)
            n = int(off[-1])
            log("segmented %s, lengths up to 2^%d: generating %d x 2 values"
                % (np.dtype(dtype).name, cap.bit_length() - 1, n))
            both = to_device_chunks(torch, synth.uniform_chunks(3, 2 * n, dtype), 2 * n, tdt, dev)
            x, y = both[:n], both[n:]
            for form in ("fast", "rigorous"):
                plan = tf.SegPlan(off, tdt, True, form)
                out = torch.empty((plan.nseg, 2), dtype=plan.out_dtype, device=dev)
                ws = tf.Workspace(plan.workspace_bytes, dev)
                t, tmin = graph_time(torch, lambda: (plan.execute(x, y, out=out, ws=ws), 1)[1])
                first = out.clone()
                plan.execute(x, y, out=out, ws=ws)
                same = bool(torch.equal(first.view(torch.int8), out.view(torch.int8)))
                nbytes = 2 * n * np.dtype(dtype).itemsize
                rows.append({"dtype": np.dtype(dtype).name, "form": form, "max_len": cap,
                             "nseg": int(plan.nseg), "elements": n, "ms": round(t * 1e3, 4),
                             "ms_min": round(tmin * 1e3, 4), "bitwise_repeatable": same,
                             "gelem_s": round(n / t / 1e9, 1), "gb_s": round(nbytes / t / 1e9, 1),
                             "hbm_frac": round(nbytes / t / 1e9 / HBM_PEAK_GBS, 4),
                             "launch": plan.launch.as_dict()})
                log("  %s %s %.3f ms %.1f GB/s" % (np.dtype(dtype).name, form, t * 1e3,
                                                   nbytes / t / 1e9))
                if form == "rigorous" and cap == 1 << 20:
                    # the precision monitor over the batch's results (tau = 2^-20)
                    od = torch.from_numpy(np.asarray(off, dtype=np.int64)).to(dev)
                    fl = torch.empty(plan.nseg, dtype=torch.int32, device=dev)
                    nf = torch.empty((), dtype=torch.int64, device=dev)
                    tm, _ = graph_time(torch, lambda: (tf.monitor(out, 2.0 ** -20, offsets=od,
                                                                  flags=fl, nflagged=nf), 1)[1])
                    rows[-1]["monitor_us"] = round(tm * 1e6, 2)
                    rows[-1]["monitor_flagged"] = int(nf.item())
                plan.close()
            del both, x, y
            torch.cuda.empty_cache()
    print(json.dumps({"workload": "segmented twofold dot, 20,000 log-uniform segments in "
                                  "[1, 2^20] (and the 2^17-capped variant), seed 3",
                      "peak_gb_s": HBM_PEAK_GBS, "device": device_info(torch, dev),
                      "rows": rows}), flush=True)


def probes(torch, tf, dev):
    """The instruments: the read probe (the paper's read1/read2) streams 1 GiB
    (and a second 1 GiB) with the reductions' 16-byte non-temporal loads;
    the compute probe (its p-functions) runs each form's step on
    register-resident items, no memory traffic. Their ratio is each form's
    arithmetic headroom over the HBM roofline. One JSON line."""
    import numpy as np

    rows = {"read": [], "compute": []}
    nbytes = 1 << 30
    x = torch.empty(nbytes // 4, dtype=torch.int32, device=dev).random_()
    y = torch.empty(nbytes // 4, dtype=torch.int32, device=dev).random_()
    for name, yy, tot in (("read1", None, nbytes), ("read2", y, 2 * nbytes)):
        for bt, u, gb in ((256, 2, 512), (256, 4, 256), (256, 8, 256), (512, 2, 256),
                          (512, 4, 256), (1024, 4, 256), (256, 4, 1024), (256, 8, 512)):
            lc = tf.Launch(bt, u, gb, 0, 0)
            sink = torch.empty(gb, dtype=torch.int64, device=dev)
            t, tmin = graph_time(torch, lambda: (tf.probe_read(x, yy, lc, sink), 1)[1], reps=20)
            rows["read"].append({"probe": name, "launch": [bt, u, gb], "us": round(t * 1e6, 2),
                                 "gb_s": round(tot / t / 1e9, 1),
                                 "hbm_frac": round(tot / t / 1e9 / HBM_PEAK_GBS, 4)})
            log("  %s %s %.1f GB/s" % (name, (bt, u, gb), tot / t / 1e9))
    del x, y
    torch.cuda.empty_cache()
    bt, gb, iters = 256, 2048, 2048
    lc = tf.Launch(bt, 4, gb, 0, 0)
    sink = torch.empty(2 * bt * gb, dtype=torch.float64, device=dev)
    forms = ("plain", "fast", "rigorous", "kahan", "wide")
    for dtype, tdt in ((np.float32, torch.float32), (np.float64, torch.float64)):
        seed = (torch.rand(64, dtype=tdt, device=dev) - 0.5)
        W = 16 // np.dtype(dtype).itemsize
        items = bt * gb * iters * 4 * W
        for op in ("sum", "dot"):
            extra = ("fast_rounded", "rigorous_rounded") if op == "dot" else ()
            if dtype == np.float32:
                extra += ("mixed",)
            for form in forms + extra:
                t, _ = graph_time(torch, lambda: (tf.probe_compute(seed, op == "dot", form, iters,
                                                                   lc, sink), 1)[1], reps=10)
                gelem = items / t / 1e9
                roof = HBM_PEAK_GBS / (np.dtype(dtype).itemsize * (2 if op == "dot" else 1))
                rows["compute"].append({"dtype": np.dtype(dtype).name, "op": op, "form": form,
                                        "gelem_s": round(gelem, 1),
                                        "over_hbm_roofline": round(gelem / roof, 2)})
                log("  compute %s %s %-16s %8.1f Gelem/s (%.1fx the HBM roofline)"
                    % (np.dtype(dtype).name, op, form, gelem, gelem / roof))
    print(json.dumps({"workload": "probes: read1/read2 over 1 GiB arrays, compute-only steps",
                      "device": device_info(torch, dev), "peak_gb_s": HBM_PEAK_GBS,
                      "rows": rows}), flush=True)


def calibrate_copy(torch, dev):
    """A plain device copy of 256 MiB, five times: its FETCH_SIZE and
    WRITE_SIZE counters per dispatch calibrate the ones of the reductions."""
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device=dev).uniform_(-1, 1)
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": COPY_BYTES,
                      "bytes_written": COPY_BYTES, "dispatches": 5}), flush=True)


KERNEL_SOURCES = ("eft.hpp", "kernels.hpp", "host_common.hpp", "batch.hip", "tuned_table.inc")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_illcond_batch_n2e24.json")


def kernel_sources_sha256():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1401_0248_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    """HBM bytes per dominant call from the committed counter summary, or
    None if the kernels changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256") != kernel_sources_sha256():
        return None
    return t.get("traffic_bytes_per_call")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--workload", choices=("illcond", "sweep", "segmented", "precision", "probes"),
                    default="illcond",
                    help="illcond: the headline line (default); sweep: the roofline sweep of "
                         "every form at 4096, 2^20 and 1 GiB per vector; segmented: the "
                         "20,000-segment batch; precision: binary32 twofold against binary64 "
                         "plain at N=2^26; probes: the read and compute instruments")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library's reduction runs on one device "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1401_0248_amd as tf

    dev = torch.device("cuda:0")
    if args.calibrate_copy:
        calibrate_copy(torch, dev)
        return
    if args.workload == "sweep":
        roofline_sweep(torch, tf, dev)
        return
    if args.workload == "segmented":
        segmented_batch(torch, tf, dev)
        return
    if args.workload == "precision":
        precision_study(torch, tf, dev, not args.no_cpu_baseline)
        return
    if args.workload == "probes":
        probes(torch, tf, dev)
        return
    log("generating 12 ill-conditioned pairs, N=2^24")
    t0 = time.perf_counter()
    host = make_inputs()
    log("inputs ready in %.1f s; copying to the GPU" % (time.perf_counter() - t0))
    dev_in = place_inputs(torch, host, dev)
    f64 = sorted((k for k in dev_in if k[0] == np.float64), key=lambda k: k[1])
    f32 = sorted((k for k in dev_in if k[0] == np.float32), key=lambda k: k[1])
    keys = {np.float64: f64, np.float32: f32}
    # One step: the rigorous and the fast dot of every pair, 24 items of both
    # data types in one mixed batch (one launch, one combine kernel). The
    # items run in turn in the order binary64 rigorous, binary32 rigorous,
    # binary64 fast, binary32 fast, so that between two reads of one pair at
    # least 768 MiB of other pairs is read and no pair is served from the
    # 256 MB last-level cache.
    items = [(k, m) for m, ks in (("rigorous", f64), ("rigorous", f32), ("fast", f64),
                                  ("fast", f32)) for k in ks]
    calls = [(dev_in[k][0], dev_in[k][1], m) for k, m in items]
    outs = [torch.empty(2, dtype=dev_in[k][0].dtype, device=dev) for k, _ in items]
    # the batch's launch: the default of its largest item, a binary64 rigorous dot
    lc = tf.default_launch(0, 8, True, "rigorous", N)
    ws = tf.Workspace(1 << 20, dev)
    bytes_step = sum(2 * N * dev_in[k][0].element_size() for k, _ in items)

    cap = torch.cuda.Stream(dev)
    tf.batch(calls, outs=outs, ws=ws)  # eager run first: loads the library, checks the call
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cap):
        tf.batch(calls, outs=outs, ws=ws)
    stream = torch.cuda.current_stream(dev)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    # A step is nothing but the batch launch (and its combine kernel), so one
    # pair of HIP events on the launch stream around the timed steps gives
    # the average launch time; an event pair around every step would add its
    # own gaps between the launches.
    log("timing %d steps" % args.steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    ndots = len(items)
    value = ndots * N * args.steps / elapsed / 1e9
    avg = e0.elapsed_time(e1) * 1e-3 / args.steps
    achieved = bytes_step / avg / 1e9
    # every result of the last timed step against the eager run, bit for bit
    repeatable = all(torch.equal(e.view(torch.int8), o.view(torch.int8))
                     for e, o in zip(eager, outs))
    log("step %.3f ms, %.1f Gelem/s; batch launch %.1f us avg by events, %.0f GB/s"
        % (ms_step, value, avg * 1e6, achieved))

    # After the timed region, for reference: every item as a single-vector
    # call with the batch's launch (results must match the batch bit for
    # bit), and the time of the six binary64 rigorous dots as single calls.
    single = [torch.empty(2, dtype=dev_in[k][0].dtype, device=dev) for k, _ in items]
    ws1 = tf.Workspace(1 << 20, dev)
    for i, (x, y, m) in enumerate(calls):
        tf.dot(x, y, m, lc, out=single[i], ws=ws1)
    batch_same = all(torch.equal(a.view(torch.int8), b.view(torch.int8))
                     for a, b in zip(single, outs))
    f64r = [i for i, (k, m) in enumerate(items) if k[0] == np.float64 and m == "rigorous"]

    def singles():
        for i in f64r:
            tf.dot(calls[i][0], calls[i][1], "rigorous", lc, out=single[i], ws=ws1)
        return len(f64r)

    single_med, _ = graph_time(torch, singles, reps=20)
    single_gbs = 2 * N * 8 / single_med / 1e9
    log("single-vector calls: %.1f us per call, %.0f GB/s; batch == single calls: %s"
        % (single_med * 1e6, single_gbs, batch_same))

    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gelem/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "ill-conditioned twofold dot, fast+rigorous, f32 and f64, "
                               "N=2^24, target cond 1e6..1e16 (12 pairs, 24 dots per step in "
                               "one mixed batch launch, HIP-graph replay)",
                   "n": N, "pairs": len(dev_in), "dots_per_step": ndots},
        "bitwise_repeatable": repeatable,
        "batch_equals_single_calls": batch_same,
        "device": device_info(torch, dev),
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(),
                     "kernel": "the step's mixed batch: 24 twofold dots of N=2^24 (binary64 and "
                               "binary32, rigorous and fast) in one launch (batch_kernel + "
                               "batch_pass2_kernel)",
                     "launch": lc.as_dict(), "bytes_per_launch": bytes_step,
                     "avg_launch_us": round(avg * 1e6, 2),
                     "single_call": {"avg_us": round(single_med * 1e6, 2),
                                     "achieved": round(single_gbs, 1),
                                     "frac": round(single_gbs / HBM_PEAK_GBS, 4),
                                     "note": "a binary64 rigorous dot of the step as a "
                                             "single-vector call with the same launch "
                                             "(single_kernel + single_pass2_kernel), graph "
                                             "replay median per call, after the timed region"}},
    }
    if not args.no_cpu_baseline:
        gpu = gpu_results(dev_in, tf)
        log("cpu baseline leg: oracle timing and grading")
        launches = {(dt, m): tf.default_launch(0, np.dtype(dt).itemsize, True, m, N)
                    for dt in (np.float32, np.float64) for m in ("rigorous", "fast")}
        import synth
        perm_host, perm_gpu = {}, {}
        for dt in (np.float32, np.float64):
            px, py = synth.permute_pairs(synth.illcond_perm_seed(16), *host[(dt, 16)])
            perm_host[dt] = (px, py)
            xd, yd = torch.from_numpy(px).to(dev), torch.from_numpy(py).to(dev)
            for mode in ("plain", "fast", "rigorous"):
                perm_gpu[(dt, mode)] = tf.dot(xd, yd, mode).double().cpu().numpy()
            perm_gpu[(dt, "dotd")] = tf.dotd(xd, yd).cpu().numpy()
            if dt == np.float32:
                perm_gpu[(dt, "mixed")] = tf.dot_mixed(xd, yd).cpu().numpy()
        res["cpu_baseline"], res["accuracy"] = oracle_leg(host, gpu, launches, perm_host, perm_gpu)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
