"""Benchmark: twofold dot products on one MI355X. Prints one JSON line.

Default workload (the line `python bench.py` prints): the batched segmented
twofold dot, 20,000 segment pairs with log-uniform lengths in [1, 2^20]
(seed 3: 1,504,333,896 elements per pair array), uniform(-1, 1) data of
seed 3 (x, then y), binary64 and binary32, rigorous and fast. One step is
the four plan executes (binary64 rigorous, binary64 fast, binary32
rigorous, binary32 fast), each one HIP graph of the segmented tile kernel
and the per-segment combine kernel, replayed in turn. `value` is the
elements of the step (4 x 1,504,333,896) over the step's wall time.

The dominant kernel is the binary64 rigorous execute (24 GB per launch); a
pair of HIP events on the launch stream around each execute of every timed
step gives its average duration and the roofline entry (algorithmic bytes /
time against 8 TB/s); the other three executes are reported beside it.

The same line carries, as sub-objects, the other measured configurations:
the ill-conditioned dot batch (24 dots of N = 2^24 in one mixed batch
launch), the roofline rows at 1 GiB per vector with the read probe's
ceiling beside them, and the binary32 precision form (N = 2^26).

The CPU-baseline leg, the only part that runs the oracle, times the
oracle's sequential paper-order twofold dots on one host thread over the
step's segments (a bounded sample), grades every segment of every form
against the exact accumulator, and checks sampled segments bit for bit
against the order model at the timed launch.
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

SEG_COUNT = 20000
SEG_MAX_LEN = 1 << 20
SEG_SEED = 3
# the step's executes, in order: (data type name, form)
SEG_FORMS = (("float64", "rigorous"), ("float64", "fast"), ("float32", "rigorous"),
             ("float32", "fast"))
ORACLE_SAMPLE_S = 25.0  # bound on the sequential oracle's timed sample
XACC_SAMPLE_S = 3.0  # seconds of one-thread exact accumulation in the accuracy leg
MODEL_SAMPLES = 48      # segments checked bit for bit against the order model

ILLCOND_N = 1 << 24
DECADES = (6, 8, 10, 12, 14, 16)


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


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


def worker_threads():
    """Host threads for generation and grading: the cores this process may
    use, at most 16."""
    return max(1, min(16, host_info()["cores_available"] or 1))


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


def capture(torch, fn):
    """A HIP graph of fn() (captured on a side stream after one eager run)."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=torch.cuda.Stream()):
        fn()
    return g


def same_bits(torch, a, b):
    return bool(torch.equal(a.view(torch.int8), b.view(torch.int8)))


# ---- the default line: the 20,000-segment batch ----------------------------

def seg_inputs(np, synth):
    """Offsets and the host data of both types: per type one array of
    2 x n values (x, then y, one stream of seed 3)."""
    lengths = synth.segment_lengths(SEG_SEED, SEG_COUNT, max_len=SEG_MAX_LEN)
    off = synth.offsets_from_lengths(lengths)
    n = int(off[-1])
    host = {}
    for name, dt in (("float64", np.float64), ("float32", np.float32)):
        t0 = time.perf_counter()
        host[name] = synth.uniform_fill(SEG_SEED, 2 * n, dt, nthreads=worker_threads())
        log("generated %s: 2 x %d values in %.1f s" % (name, n, time.perf_counter() - t0))
    return off, n, host


def seg_headline(args, np, torch, tf, dev):
    """The timed step. Returns the result dict and what the oracle leg needs."""
    import synth
    off, n, host = seg_inputs(np, synth)
    tdt = {"float64": torch.float64, "float32": torch.float32}
    dev_in = {}
    for name, h in host.items():
        t0 = time.perf_counter()
        both = torch.from_numpy(h).to(dev)
        dev_in[name] = (both[:n], both[n:])
        log("copied %s to the GPU in %.1f s" % (name, time.perf_counter() - t0))
    execs = []
    for name, form in SEG_FORMS:
        plan = tf.SegPlan(off, tdt[name], True, form)
        out = torch.empty((plan.nseg, 2), dtype=plan.out_dtype, device=dev)
        ws = tf.Workspace(plan.workspace_bytes, dev)
        x, y = dev_in[name]

        def run(plan=plan, x=x, y=y, out=out, ws=ws):
            plan.execute(x, y, out=out, ws=ws)

        execs.append({"name": name, "form": form, "plan": plan, "out": out, "ws": ws, "run": run,
                      "bytes": 2 * n * (8 if name == "float64" else 4)})
    eager = []
    for e in execs:
        e["run"]()
    torch.cuda.synchronize()
    eager = [e["out"].clone() for e in execs]
    graphs = [capture(torch, e["run"]) for e in execs]
    stream = torch.cuda.current_stream(dev)

    log("warmup %d" % args.warmup)
    for _ in range(args.warmup):
        for g in graphs:
            g.replay()
    torch.cuda.synchronize()
    log("timing %d steps" % args.steps)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(len(graphs) + 1)]
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        evs[s][0].record(stream)
        for i, g in enumerate(graphs):
            g.replay()
            evs[s][i + 1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_step = 1e3 * elapsed / args.steps
    elems_step = len(execs) * n
    value = elems_step * args.steps / elapsed / 1e9
    per_form = []
    for i, e in enumerate(execs):
        avg = sum(evs[s][i].elapsed_time(evs[s][i + 1]) for s in range(args.steps)) \
            * 1e-3 / args.steps
        gbs = e["bytes"] / avg / 1e9
        per_form.append({"dtype": e["name"], "form": e["form"], "avg_execute_us": round(avg * 1e6, 2),
                         "gelem_s": round(n / avg / 1e9, 2), "achieved_gb_s": round(gbs, 1),
                         "frac": round(gbs / HBM_PEAK_GBS, 4),
                         "launch": e["plan"].launch.as_dict()})
    ev_step = evs[0][0].elapsed_time(evs[-1][-1]) * 1e-3 / args.steps
    repeatable = all(same_bits(torch, a, e["out"]) for a, e in zip(eager, execs))
    log("step %.3f ms, %.1f Gelem/s; %s" % (ms_step, value, ", ".join(
        "%s %s %.1f us %.0f GB/s" % (p["dtype"], p["form"], p["avg_execute_us"], p["achieved_gb_s"])
        for p in per_form)))
    dom = per_form[0]  # binary64 rigorous: the most bytes per launch
    res = {
        "metric": METRIC, "value": round(value, 2), "unit": "Gelem/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batched segmented twofold dot: 20,000 segment pairs, lengths "
                               "log-uniform in [1, 2^20] (seed 3), uniform(-1,1) data (seed 3), "
                               "binary64 and binary32, rigorous and fast: 4 plan executes per "
                               "step, each a HIP-graph replay of one persistent tile kernel and "
                               "the per-segment combine",
                   "nseg": SEG_COUNT, "elements_per_dot": n, "dots_per_step": len(execs),
                   "elements_per_step": elems_step},
        "bitwise_repeatable": repeatable,
        "device": device_info(torch, dev),
        "roofline": {"bound": "hbm", "achieved": dom["achieved_gb_s"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": dom["frac"], "traffic": measured_traffic(SEG_TRAFFIC),
                     "kernel": "binary64 rigorous segmented dot execute: seg_kernel "
                               "(persistent tile kernel) + seg_pass2_kernel (per-segment "
                               "combine), 20,000 segments",
                     "launch": dom["launch"], "bytes_per_launch": execs[0]["bytes"],
                     "avg_launch_us": dom["avg_execute_us"],
                     "timing": "HIP events on the launch stream around each execute of every "
                               "timed step"},
        "per_form": per_form,
        "step_by_events_ms": round(ev_step * 1e3, 4),
    }
    state = {"off": off, "n": n, "host": host, "execs": execs}
    del dev_in
    return res, state


def seg_oracle_leg(np, torch, state):
    """cpu_baseline, grading and sampled order-model parity of the headline."""
    import oracle
    from oracle import bounds

    off, n, host, execs = state["off"], state["n"], state["host"], state["execs"]
    nseg = off.size - 1
    xs = {k: (v[:n], v[n:]) for k, v in host.items()}
    outs = [e["out"].double().cpu().numpy() for e in execs]

    # (1) the sequential oracle on one host thread, segments in the step's
    # order, for at most ORACLE_SAMPLE_S seconds
    t0 = time.perf_counter()
    done_elems, done_segs = 0, []
    for i, e in enumerate(execs):
        x, y = xs[e["name"]]
        kind = "dott" if e["form"] == "rigorous" else "dottf"
        s = 0
        while s < nseg and time.perf_counter() - t0 < ORACLE_SAMPLE_S:
            a, b = int(off[s]), int(off[s + 1])
            oracle.seq(kind, x[a:b], y[a:b])
            done_elems += b - a
            s += 1
        done_segs.append(s)
        if time.perf_counter() - t0 >= ORACLE_SAMPLE_S:
            break
    dt_s = time.perf_counter() - t0
    forms_done = ["%s %s: %d of %d segments" % (e["name"], e["form"], c, nseg)
                  for e, c in zip(execs, done_segs)]
    base = {"value": round(done_elems / dt_s / 1e9, 4), "unit": "Gelem/s", "cores": 1,
            "kind": "oracle",
            "sample": "sequential twofold dots (paper order, FMA remainder; rigorous and fast) of "
                      "the step's segments in its order on one host thread, stopped after "
                      "%.0f s: %s; %d elements in %.1f s" % (ORACLE_SAMPLE_S,
                                                             "; ".join(forms_done), done_elems, dt_s),
            "host": host_info()}

    # (2) the exact accumulator alone, on one host thread, over the first
    # binary64 segments (a bounded sample), for its rate beside the
    # all-thread grading below
    lens = np.diff(off)
    x64, y64 = xs["float64"]
    t1 = time.perf_counter()
    one_elems, one_segs = 0, 0
    while one_segs < nseg and time.perf_counter() - t1 < XACC_SAMPLE_S:
        a, b = int(off[one_segs]), int(off[one_segs + 1])
        oracle.Exact(x64[a:b], y64[a:b], nthreads=1)
        one_elems += b - a
        one_segs += 1
    one_s = time.perf_counter() - t1

    # (3) every segment of every form against the exact accumulator
    t0 = time.perf_counter()

    def exact_seg(args):
        name, s = args
        x, y = xs[name]
        a, b = int(off[s]), int(off[s + 1])
        ex = oracle.Exact(x[a:b], y[a:b], nthreads=1)
        row = []
        for i, e in enumerate(execs):
            if e["name"] != name:
                continue
            v, er = outs[i][s]
            row.append((i, abs(ex.diff(v, er)), abs(ex.diff(v))))
        return name, s, ex.A, row

    D = np.zeros((len(execs), nseg))
    Dv = np.zeros((len(execs), nseg))
    A = {k: np.zeros(nseg) for k in xs}
    jobs = [(k, s) for k in xs for s in range(nseg)]
    with ThreadPoolExecutor(max_workers=worker_threads()) as ex:
        for name, s, a_s, row in ex.map(exact_seg, jobs, chunksize=64):
            A[name][s] = a_s
            for i, d, dv in row:
                D[i, s] = d
                Dv[i, s] = dv
    grade_s = time.perf_counter() - t0
    acc = {"measure": "per segment: |v + e - S| / sum|x y| (median, max), largest |v + e - S| "
                      "over 4 L u^2 sum|x y| (L the segment's length) and over the proven bound "
                      "of the segment's reduction tree at the timed launch, segments above "
                      "4 L u^2 sum|x y|; value_median: median |v - S| / sum|x y|",
           "segments_graded": nseg, "grading_s": round(grade_s, 1),
           "exact_accumulator": {
               "all_threads_gelem_s": round(sum(len(v[0]) for v in xs.values()) / grade_s / 1e9, 4),
               "threads": worker_threads(),
               "one_thread_gelem_s": round(one_elems / one_s / 1e9, 4) if one_s > 0 else None,
               "one_thread_sample": "the first %d binary64 segments, %d dot elements, in %.2f s"
                                    % (one_segs, one_elems, one_s),
               "note": "all threads: every segment of both types, diffs against every execute "
                       "included"}}
    for i, e in enumerate(execs):
        dt = np.float64 if e["name"] == "float64" else np.float32
        u = bounds.unit_roundoff(dt)
        a_ = A[e["name"]]
        ok = a_ > 0
        rel = D[i][ok] / a_[ok]
        tol = 4.0 * lens[ok] * u * u * a_[ok]
        ts = e["plan"].launch.tile_elems
        if e["form"] == "rigorous":
            tb = np.array([bounds.segment_bound(dt, int(L), ts, float(aa))
                           for L, aa in zip(lens[ok], a_[ok])])
            over_tree = float("%.3g" % float(np.max(D[i][ok] / tb)))
        else:
            over_tree = None
        acc["%s_%s" % (e["name"], e["form"])] = {
            "median": float("%.3g" % float(np.median(rel))), "max": float("%.3g" % float(rel.max())),
            "max_over_4Lu2_bound": float("%.3g" % float(np.max(D[i][ok] / tol))),
            "segments_over_4Lu2_bound": int(np.sum(D[i][ok] > tol)),
            "max_over_tree_bound": over_tree,
            "value_median": float("%.3g" % float(np.median(Dv[i][ok] / a_[ok])))}

    # (3) sampled segments bit for bit against the order model at the timed launch
    rng = np.random.default_rng(7)
    pick = sorted(set([int(np.argmax(lens)), int(np.argmin(lens)), nseg - 1]
                      + [int(v) for v in rng.choice(nseg, MODEL_SAMPLES, replace=False)]))
    mism = 0
    for i, e in enumerate(execs):
        x, y = xs[e["name"]]
        lc = e["plan"].launch
        W = 16 // x.itemsize
        for s in pick:
            a, b = int(off[s]), int(off[s + 1])
            want = oracle.model_seg(e["form"], x[a:b], np.array([0, b - a]), y[a:b],
                                    x_misalign=a % W, unroll=lc.unroll, tile_elems=lc.tile_elems)
            got = outs[i][s]
            if not (np.array(want[0], dtype=np.float64).view(np.uint64)
                    == np.array(got, dtype=np.float64).view(np.uint64)).all():
                mism += 1
    parity = {"segments_checked_per_form": len(pick), "forms": len(execs), "mismatches": mism,
              "against": "the order model (oracle) at each execute's launch"}
    return base, acc, parity


# ---- sub-object: the ill-conditioned dot batch -----------------------------

def make_illcond(np, synth):
    jobs = [(dt, d) for dt in (np.float32, np.float64) for d in DECADES]

    def one(job):
        dt, d = job
        return job, synth.illcond_dot(synth.illcond_seed(d), ILLCOND_N, 10.0 ** d, dt)

    with ThreadPoolExecutor(max_workers=min(12, worker_threads())) as ex:
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


def illcond_batch(np, torch, tf, dev, steps, warmup, with_oracle):
    """24 dots of N = 2^24 (binary32 and binary64 pairs of target
    conditions 1e6..1e16, rigorous and fast) in one mixed batch launch per
    step; the timed results are graded against the exact sum."""
    import synth
    log("ill-conditioned batch: generating 12 pairs, N=2^24")
    host = make_illcond(np, synth)
    dev_in = place_inputs(torch, host, dev)
    keys = {dt: sorted((k for k in dev_in if k[0] == dt), key=lambda k: k[1])
            for dt in (np.float64, np.float32)}
    # binary64 rigorous, binary32 rigorous, binary64 fast, binary32 fast: at
    # least 768 MiB of other pairs between two reads of one pair, so none is
    # served from the 256 MB last-level cache
    items = [(k, m) for m, dt in (("rigorous", np.float64), ("rigorous", np.float32),
                                  ("fast", np.float64), ("fast", np.float32)) for k in keys[dt]]
    calls = [(dev_in[k][0], dev_in[k][1], m) for k, m in items]
    outs = [torch.empty(2, dtype=dev_in[k][0].dtype, device=dev) for k, _ in items]
    lc = tf.default_launch(0, 8, True, "rigorous", ILLCOND_N)
    ws = tf.Workspace(1 << 20, dev)
    bytes_step = sum(2 * ILLCOND_N * dev_in[k][0].element_size() for k, _ in items)
    g = capture(torch, lambda: tf.batch(calls, lc, outs=outs, ws=ws))
    eager = [o.clone() for o in outs]
    stream = torch.cuda.current_stream(dev)
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        g.replay()
    e1.record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    avg = e0.elapsed_time(e1) * 1e-3 / steps
    repeatable = all(same_bits(torch, a, b) for a, b in zip(eager, outs))
    single = [torch.empty(2, dtype=dev_in[k][0].dtype, device=dev) for k, _ in items]
    ws1 = tf.Workspace(1 << 20, dev)
    for i, (x, y, m) in enumerate(calls):
        tf.dot(x, y, m, lc, out=single[i], ws=ws1)
    batch_same = all(same_bits(torch, a, b) for a, b in zip(single, outs))
    f64r = [i for i, (k, m) in enumerate(items) if k[0] == np.float64 and m == "rigorous"]

    def singles():
        for i in f64r:
            tf.dot(calls[i][0], calls[i][1], "rigorous", lc, out=single[i], ws=ws1)
        return len(f64r)

    single_med, _ = graph_time(torch, singles, reps=20)
    single_gbs = 2 * ILLCOND_N * 8 / single_med / 1e9
    achieved = bytes_step / avg / 1e9
    log("ill-conditioned batch: %.1f us per launch, %.0f GB/s; single call %.1f us"
        % (avg * 1e6, achieved, single_med * 1e6))
    res = {"workload": "ill-conditioned twofold dot, fast+rigorous, binary32 and binary64, "
                       "N=2^24, target cond 1e6..1e16 (12 pairs, 24 dots in one mixed batch "
                       "launch per step, HIP-graph replay)",
           "steps": steps, "gelem_s": round(len(items) * ILLCOND_N * steps / elapsed / 1e9, 2),
           "ms_per_step": round(1e3 * elapsed / steps, 4),
           "avg_launch_us": round(avg * 1e6, 2), "achieved_gb_s": round(achieved, 1),
           "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(ILLCOND_TRAFFIC),
           "launch": lc.as_dict(), "bytes_per_launch": bytes_step,
           "bitwise_repeatable": repeatable, "batch_equals_single_calls": batch_same,
           "single_call": {"avg_us": round(single_med * 1e6, 2), "achieved_gb_s": round(single_gbs, 1),
                           "frac": round(single_gbs / HBM_PEAK_GBS, 4),
                           "note": "a binary64 rigorous dot of the batch as a single-vector call "
                                   "with the same launch (single_kernel + single_pass2_kernel), "
                                   "graph replay median per call"}}
    if with_oracle:
        res["accuracy_timed"] = grade_illcond_timed(np, host, items, outs, lc)
        res["default_launch_forms"] = illcond_default_forms(np, torch, tf, dev, host, dev_in)
    del dev_in
    return res


def grade_illcond_timed(np, host, items, outs, lc):
    """The pairs of the last timed replay, graded against the exact sum with
    the batch's own launch: |D| / sum|x y|, and for the rigorous form the
    largest |D| over the proven bound of that launch's tree and over
    4 N u^2 sum|x y|."""
    import oracle
    from oracle import bounds
    rows = {}
    exact = {}
    for (k, m), o in zip(items, outs):
        dt, d = k
        if k not in exact:
            exact[k] = oracle.Exact(*host[k])
        ex = exact[k]
        v, e = (float(t) for t in o.double().cpu().numpy())
        D = abs(ex.diff(v, e))
        key = "%s_%s" % ("f32" if dt == np.float32 else "f64", m)
        rows.setdefault(key, []).append(D / ex.A)
        if m == "rigorous":
            u = bounds.unit_roundoff(dt)
            tb = bounds.single_bound(dt, ILLCOND_N, lc.block_threads, lc.unroll, lc.grid_blocks,
                                     ex.A)
            rows.setdefault(key + "_over_tree_bound", []).append(D / tb)
            rows.setdefault(key + "_over_4Nu2_bound", []).append(D / (4 * ILLCOND_N * u * u * ex.A))
        if m == "rigorous" and dt == np.float64:
            rows.setdefault("cond_f64", []).append(2 * ex.A / abs(ex.S) if ex.S else float("inf"))
        if m == "rigorous" and dt == np.float32:
            rows.setdefault("cond_f32", []).append(2 * ex.A / abs(ex.S) if ex.S else float("inf"))
    acc = {"measure": "the timed batch's pairs (launch %s): median over conditions of "
                      "|v + e - S| / sum|x y|; *_bound: the largest |v + e - S| over the bound"
                      % lc.as_dict()}
    for k, v in rows.items():
        if k.startswith("cond_"):
            acc[k] = ["%.3g" % c for c in v]
        elif k.endswith("_bound"):
            acc[k] = float("%.3g" % max(v))
        else:
            acc[k] = float("%.3g" % float(np.median(v)))
    return acc


def illcond_default_forms(np, torch, tf, dev, host, dev_in):
    """Every form as its own single-vector call with its default launch
    (outside the timed batch): median |v + e - S| / sum|x y| over the
    conditions, plain, fast, rigorous, the wider accumulator and for
    binary32 data the mixed form."""
    import oracle
    rows = {}
    for k, (xd, yd) in dev_in.items():
        dt = k[0]
        ex = oracle.Exact(*host[k])
        key = "f32" if dt == np.float32 else "f64"
        got = {m: tf.dot(xd, yd, m).double().cpu().numpy() for m in ("plain", "fast", "rigorous")}
        got["wide"] = tf.dotd(xd, yd).cpu().numpy()
        if dt == np.float32:
            got["mixed"] = tf.dot_mixed(xd, yd).cpu().numpy()
        for m, p in got.items():
            rows.setdefault("%s_%s" % (key, m), []).append(abs(ex.diff(p[0], p[1])) / ex.A)
    out = {"measure": "default launches, median over conditions of |v + e - S| / sum|x y| "
                      "(wide: binary64 sum of binary32 data, double-word for binary64 data)"}
    for k, v in rows.items():
        out[k] = float("%.3g" % float(np.median(v)))
    return out


# ---- sub-object: 1 GiB per vector, with the read probe beside -------------

PROBE_LAUNCHES = ((256, 2, 256), (256, 4, 256), (256, 8, 256), (256, 4, 512), (256, 8, 512),
                  (512, 4, 256), (512, 8, 256), (1024, 4, 256), (256, 2, 1024), (512, 2, 512))


def probe_rate(torch, tf, x, y, lc):
    """GB/s of the read probe over x (and y) with launch lc (median over 10
    graph replays of 4 calls, per call, as the rows it stands beside)."""
    nbytes = x.numel() * x.element_size()
    sink = torch.empty(lc.grid_blocks, dtype=torch.int64, device=x.device)

    def calls():
        for _ in range(4):
            tf.probe_read(x, y, lc, sink)
        return 4

    t, _ = graph_time(torch, calls, reps=10)
    return nbytes * (2 if y is not None else 1) / t / 1e9


def roofline_1gib(np, torch, tf, dev):
    """Plain, fast and rigorous sum and dot at 1 GiB per vector (binary32
    N = 2^28, binary64 N = 2^27), uniform(-1, 1) data of seed 1, tuned
    default launches, HIP-graph replay (4 calls per replay); each row beside
    the read probe over the same bytes with the row's own launch, and the
    best probe rate over a set of launches."""
    import synth
    rows, probes = [], {}
    for dtype, tdt in ((np.float32, torch.float32), (np.float64, torch.float64)):
        size = np.dtype(dtype).itemsize
        n = (1 << 30) // size
        both = torch.from_numpy(synth.uniform_fill(1, 2 * n, dtype, nthreads=worker_threads())).to(dev)
        x, y = both[:n], both[n:]
        for two in (False, True):
            key = "%s_%s" % (np.dtype(dtype).name, "read2" if two else "read1")
            best = max((probe_rate(torch, tf, x, y if two else None, tf.Launch(bt, u, gb, 0, 0)),
                        (bt, u, gb)) for bt, u, gb in PROBE_LAUNCHES)
            probes[key] = {"best_gb_s": round(best[0], 1), "best_launch": list(best[1]),
                           "frac": round(best[0] / HBM_PEAK_GBS, 4)}
        for op in ("sum", "dot"):
            for form in ("plain", "fast", "rigorous"):
                lc = tf.default_launch(0, size, op == "dot", form, n)
                out = torch.empty(2, dtype=tdt, device=dev)
                ws = tf.Workspace(tf._lib.load().twofold_workspace_bytes_single(
                    size, op == "dot", tf.mode_id(form), n, None), dev)

                def calls():
                    for _ in range(4):
                        if op == "dot":
                            tf.dot(x, y, form, out=out, ws=ws)
                        else:
                            tf.sum(x, form, out=out, ws=ws)
                    return 4

                t, tmin = graph_time(torch, calls, reps=10)
                nbytes = n * size * (2 if op == "dot" else 1)
                gbs = nbytes / t / 1e9
                probe_same = probe_rate(torch, tf, x, y if op == "dot" else None, lc)
                pk = "%s_%s" % (np.dtype(dtype).name, "read2" if op == "dot" else "read1")
                rows.append({"dtype": np.dtype(dtype).name, "op": op, "form": form, "n": n,
                             "us": round(t * 1e6, 2), "gelem_s": round(n / t / 1e9, 1),
                             "gb_s": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                             "launch": [lc.block_threads, lc.unroll, lc.grid_blocks],
                             "probe_same_launch_gb_s": round(probe_same, 1),
                             "frac_of_probe_same_launch": round(gbs / probe_same, 4),
                             "frac_of_best_probe": round(gbs / probes[pk]["best_gb_s"], 4)})
                log("1 GiB %s %s %-8s %8.1f us %7.1f GB/s (%.3f), probe same launch %.1f GB/s"
                    % (np.dtype(dtype).name, op, form, t * 1e6, gbs, gbs / HBM_PEAK_GBS, probe_same))
        del both, x, y
        torch.cuda.empty_cache()
    return {"workload": "roofline at 1 GiB per vector: plain, fast, rigorous sum and dot, binary32 "
                        "N=2^28 and binary64 N=2^27, uniform(-1,1) seed 1, tuned default launches; "
                        "us = median over 10 graph replays of 4 calls, per call",
            "rows": rows, "read_probe": probes,
            "probe_note": "the read probe runs the single-vector kernel's own lane loop with a "
                          "bit-OR in place of the summation step (twofold_probe_read)"}


# ---- sub-object: the binary32 precision form --------------------------------

def precision_study(np, torch, tf, dev, with_oracle):
    """The binary32 precision form: N = 2^26 binary32 pairs x = m 2^k, y
    likewise (m uniform(-1, 1), k uniform integer in [-20, 20], seed 2).
    Times the binary32 plain, fast and rigorous twofold dots, the mixed
    form (binary32 rigorous value, binary64 error term), the binary64 plain
    dot of the same binary32 data (dotd) and the binary64 plain and
    rigorous dots over a binary64 copy (twice the bytes), HIP-graph replay.
    Its oracle part grades every result against the exact accumulator and
    times the oracle's sequential rigorous dot on the same data."""
    import synth

    n = 1 << 26
    log("precision form: generating N=2^26 scaled binary32 pairs")
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
    res = {"workload": "precision form: binary32 twofold vs binary64 plain, N=2^26, "
                       "x, y = uniform(-1,1) * 2^k, k in [-20, 20], seed 2",
           "n": n, "rows": rows}
    if with_oracle:
        import oracle
        ex = oracle.Exact(x, y)
        for r in rows:
            v, e = results[r["form"]]
            r["err_rel"] = float("%.3g" % (abs(ex.diff(v, e)) / ex.A))
        t0 = time.perf_counter()
        oracle.seq("dott", x, y)
        dt_s = time.perf_counter() - t0
        res["cpu_baseline"] = {"value": round(n / dt_s / 1e9, 4), "unit": "Gelem/s", "cores": 1,
                               "kind": "oracle", "sample": "sequential rigorous twofold dot "
                               "(paper order, FMA remainder) of the whole pair, %.1f s" % dt_s}
        res["err_measure"] = "|v + e - S| / sum|x y| against the exact accumulator"
    del xd, yd, x64, y64
    torch.cuda.empty_cache()
    return res


# ---- detailed workloads (their own JSON lines) --------------------------------

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


FORMS = ("plain", "fast", "rigorous")


def roofline_sweep(np, torch, tf, dev):
    """Every form of sum and dot (plain, fast, rigorous, Kahan, the wide
    accumulator, for binary32 data the mixed form, and for dots the paper's
    rounded-product fast and rigorous forms), binary32 and binary64, at
    N = 4096, 2^20 and 1 GiB per vector, uniform(-1, 1) data of seed 1,
    tuned default launches, HIP-graph replay: the method comparison of the
    paper's Table 1 on one MI355X. One JSON line."""
    import synth

    rows = []
    scrub = torch.zeros(SCRUB_BYTES // 4, dtype=torch.float32, device=dev)
    for dtype, tdt in ((np.float32, torch.float32), (np.float64, torch.float64)):
        size = np.dtype(dtype).itemsize
        for n in (4096, 1 << 20, (1 << 30) // size):
            log("sweep %s n=%d" % (np.dtype(dtype).name, n))
            both = torch.from_numpy(synth.uniform_fill(1, 2 * n, dtype,
                                                       nthreads=worker_threads())).to(dev)
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
                    row["bitwise_repeatable"] = same_bits(torch, first, o)
                    rows.append(row)
                    log("  %s %-16s %10.2f us %8.1f GB/s" % (op, form, t * 1e6, nbytes / t / 1e9))
            del both, x, y
            torch.cuda.empty_cache()
    print(json.dumps({"device": device_info(torch, dev),
                      "workload": "roofline sweep, uniform(-1,1) seed 1, tuned default launches; "
                                  "us = median over 30 graph replays of 50 calls (4 at 1 GiB) "
                                  "per call, warm; us_cold = one call after a 512 MiB scrub",
                      "peak_gb_s": HBM_PEAK_GBS, "rows": rows}), flush=True)


def segmented_batch(np, torch, tf, dev):
    """20,000 segment pairs with log-uniform lengths in [1, 2^20] (seed 3,
    1,504,333,896 elements), the secondary variant capped at 2^17
    (221,217,512 elements), and a batch of short segments (1,000,000
    log-uniform in [1, 2^9], seed 9: the launch rows for short segments);
    uniform(-1, 1) data of seed 3 (x, then y), binary32 and binary64, fast
    and rigorous dots through plans with the tuned default launch,
    HIP-graph replay, plus the precision monitor over the rigorous results.
    One JSON line."""
    import synth

    rows = []
    for dtype, tdt in ((np.float32, torch.float32), (np.float64, torch.float64)):
        for cap in (1 << 20, 1 << 17, 1 << 9):
            if cap == 1 << 9:
                lengths = synth.segment_lengths(9, 1000000, max_len=cap)
            else:
                lengths = synth.segment_lengths(3, 20000, max_len=cap)
            off = synth.offsets_from_lengths(lengths)
            n = int(off[-1])
            log("segmented %s, lengths up to 2^%d: generating %d x 2 values"
                % (np.dtype(dtype).name, cap.bit_length() - 1, n))
            both = torch.from_numpy(synth.uniform_fill(3, 2 * n, dtype,
                                                       nthreads=worker_threads())).to(dev)
            x, y = both[:n], both[n:]
            for form in ("fast", "rigorous"):
                plan = tf.SegPlan(off, tdt, True, form)
                out = torch.empty((plan.nseg, 2), dtype=plan.out_dtype, device=dev)
                ws = tf.Workspace(plan.workspace_bytes, dev)
                t, tmin = graph_time(torch, lambda: (plan.execute(x, y, out=out, ws=ws), 1)[1])
                first = out.clone()
                plan.execute(x, y, out=out, ws=ws)
                same = same_bits(torch, first, out)
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
                                  "[1, 2^20] (and the 2^17-capped variant), seed 3; "
                                  "1,000,000 short segments in [1, 2^9], seed 9",
                      "peak_gb_s": HBM_PEAK_GBS, "device": device_info(torch, dev),
                      "rows": rows}), flush=True)


def probes(np, torch, tf, dev):
    """The instruments: the read probe (the paper's read1/read2) streams 1 GiB
    (and a second 1 GiB) through the single-vector lane loop over a set of
    launches; the compute probe (its p-functions) runs each form's step on
    register-resident items, no memory traffic. Their ratio is each form's
    arithmetic headroom over the HBM roofline. One JSON line."""
    rows = {"read": [], "compute": []}
    nbytes = 1 << 30
    x = torch.empty(nbytes // 4, dtype=torch.int32, device=dev).random_()
    y = torch.empty(nbytes // 4, dtype=torch.int32, device=dev).random_()
    for name, yy in (("read1", None), ("read2", y)):
        for bt, u, gb in PROBE_LAUNCHES:
            g = probe_rate(torch, tf, x, yy, tf.Launch(bt, u, gb, 0, 0))
            rows["read"].append({"probe": name, "launch": [bt, u, gb], "gb_s": round(g, 1),
                                 "hbm_frac": round(g / HBM_PEAK_GBS, 4)})
            log("  %s %s %.1f GB/s" % (name, (bt, u, gb), g))
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


def single_calls(np, torch, tf, dev):
    """Per-call cost of the single-vector path: the binary64 rigorous dot of
    N = 2^24 uniform(-1, 1) pairs (seed 0) at its default launch, 50 calls
    back to back, as one HIP-graph replay and as eager launches; per-call
    time by events around all 50. Under a kernel trace the dispatches show
    how a call's time splits into the reduce kernel, the gap before the
    combine kernel, the combine and the gap before the next call. One JSON
    line."""
    import synth
    n = 1 << 24
    both = torch.from_numpy(synth.uniform_fill(0, 2 * n, np.float64,
                                               nthreads=worker_threads())).to(dev)
    x, y = both[:n], both[n:]
    lc = tf.default_launch(0, 8, True, "rigorous", n)
    out = torch.empty(2, dtype=torch.float64, device=dev)
    ws = tf.Workspace(1 << 20, dev)
    calls = 50

    def run():
        for _ in range(calls):
            tf.dot(x, y, "rigorous", lc, out=out, ws=ws)
        return calls

    t_graph, t_graph_min = graph_time(torch, run, reps=10)
    st = torch.cuda.current_stream(dev)
    ts = []
    for _ in range(10):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        run()
        e1.record(st)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) * 1e-3 / calls)
    import statistics
    t_eager = statistics.median(ts)
    nbytes = 2 * n * 8
    res = {"workload": "single-vector binary64 rigorous dot, N=2^24 (256 MiB per call), "
                       "50 calls back to back", "launch": lc.as_dict(),
           "graph_us_per_call": round(t_graph * 1e6, 2),
           "graph_frac": round(nbytes / t_graph / 1e9 / HBM_PEAK_GBS, 4),
           "eager_us_per_call": round(t_eager * 1e6, 2),
           "eager_frac": round(nbytes / t_eager / 1e9 / HBM_PEAK_GBS, 4),
           "device": device_info(torch, dev)}
    log("single calls: graph %.2f us/call (%.3f), eager %.2f us/call (%.3f)"
        % (t_graph * 1e6, res["graph_frac"], t_eager * 1e6, res["eager_frac"]))
    print(json.dumps(res), flush=True)


COPY_BYTES = 1 << 28


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


# ---- HBM traffic from committed counter summaries -------------------------------

# (summary file, kernel sources its counters depend on)
SEG_TRAFFIC = ("traffic_segmented_dot_20000seg.json",
               ("eft.hpp", "kernels.hpp", "host_common.hpp", "segmented.hip", "tuned_table.inc"))
ILLCOND_TRAFFIC = ("traffic_illcond_batch_n2e24.json",
                   ("eft.hpp", "kernels.hpp", "host_common.hpp", "batch.hip", "tuned_table.inc"))


def kernel_sources_sha256(sources):
    import hashlib
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, "paper_1401_0248_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(which):
    """HBM bytes per dominant call from the committed counter summary, or
    None if the kernels changed since the counters were taken."""
    fname, sources = which
    try:
        with open(os.path.join(ROOT, "profiles", fname)) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_sources_sha256") != kernel_sources_sha256(sources):
        return None
    return t.get("traffic_bytes_per_call")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip every oracle part (timing, grading, order-model parity)")
    ap.add_argument("--no-sub", action="store_true",
                    help="default line only: skip the sub-objects of the other configurations")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain device copy of known size (counter calibration)")
    ap.add_argument("--workload", choices=("headline", "illcond", "sweep", "segmented",
                                           "precision", "probes", "single"),
                    default="headline",
                    help="headline: the default line (20,000-segment batch with the other "
                         "configurations as sub-objects); illcond: the ill-conditioned batch "
                         "alone; sweep: every form at 4096, 2^20 and 1 GiB per vector; "
                         "segmented: both segment batches and the monitor; precision: binary32 "
                         "twofold against binary64 plain at N=2^26; probes: the instruments; "
                         "single: the per-call cost of single-vector dots")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this library's reduction runs on one device "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1401_0248_amd as tf

    dev = torch.device("cuda:0")
    with_oracle = not args.no_cpu_baseline
    if args.calibrate_copy:
        calibrate_copy(torch, dev)
        return
    if args.workload == "sweep":
        roofline_sweep(np, torch, tf, dev)
        return
    if args.workload == "segmented":
        segmented_batch(np, torch, tf, dev)
        return
    if args.workload == "precision":
        res = precision_study(np, torch, tf, dev, with_oracle)
        res["device"] = device_info(torch, dev)
        print(json.dumps(res), flush=True)
        return
    if args.workload == "probes":
        probes(np, torch, tf, dev)
        return
    if args.workload == "single":
        single_calls(np, torch, tf, dev)
        return
    if args.workload == "illcond":
        res = illcond_batch(np, torch, tf, dev, args.steps, args.warmup, with_oracle)
        res["device"] = device_info(torch, dev)
        print(json.dumps(res), flush=True)
        return

    res, state = seg_headline(args, np, torch, tf, dev)
    for e in state["execs"]:
        e["plan"].close()
    if with_oracle:
        log("cpu baseline leg: oracle timing, grading of every segment, order-model samples")
        t0 = time.perf_counter()
        res["cpu_baseline"], res["accuracy"], res["parity_sampled"] = seg_oracle_leg(np, torch, state)
        log("cpu baseline leg done in %.1f s" % (time.perf_counter() - t0))
    state["execs"].clear()  # the device inputs and outputs go with the executes
    del state
    torch.cuda.empty_cache()
    if not args.no_sub:
        res["illcond_batch"] = illcond_batch(np, torch, tf, dev, args.steps, args.warmup,
                                             with_oracle)
        torch.cuda.empty_cache()
        res["roofline_1gib"] = roofline_1gib(np, torch, tf, dev)
        res["precision"] = precision_study(np, torch, tf, dev, with_oracle)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
