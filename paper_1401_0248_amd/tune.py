"""Autotuner for the launch table compiled into libtwofold.so.

For every (kind, dtype, op, mode) and every size bucket it times a set of
candidate launch shapes on the current GPU and keeps the fastest. Timing:
R calls captured into one HIP graph (rotating over input copies so large
inputs are not served from cache), replayed several times between HIP
events; the median replay gives the time per call.

Single vector: block_threads x unroll x max_blocks (the grid is the blocks
one round needs, capped at max_blocks). Segmented plans: block_threads x
unroll x grid_blocks x tile_elems, on log-uniform segment lengths (the
batch shape the segmented path is built for).

Writes the table as C rows (csrc/tuned_table.inc format) to --out.
The tuned values change result bits (the reduction order depends on the
launch), so the table is checked in and changed only by re-running this.

Usage: python -m paper_1401_0248_amd.tune --out tuned_table.inc [--quick]
       [--only single|seg] [--combo DTYPE,IS_DOT,MODE ...] [--bucket N_MAX ...]
       [--passes P]
With --combo (or --bucket) only those combinations (size buckets) are
timed, and the file holds only their rows, to be merged into
csrc/tuned_table.inc in place of theirs. With --passes P every
single-vector candidate is timed P times, in alternating order, and keeps
its best time.
"""
import argparse
import itertools
import os
import statistics
import sys
import time

import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1401_0248_amd as tf  # noqa: E402

MODES = {0: "plain", 1: "fast", 2: "rigorous", 3: "wide", 4: "kahan", 5: "fast_rounded",
         6: "rigorous_rounded", 7: "mixed"}
# (dtype, is_dot, mode): every form of the library (wide is binary64 for
# binary32 data and double-word for binary64 data); the rounded-product
# forms are dots only, the mixed form binary32 only
COMBOS = [(4, 0, 0), (4, 0, 1), (4, 0, 2), (4, 0, 3), (4, 0, 4),
          (8, 0, 0), (8, 0, 1), (8, 0, 2), (8, 0, 3), (8, 0, 4),
          (4, 1, 0), (4, 1, 1), (4, 1, 2), (4, 1, 3), (4, 1, 4), (4, 1, 5), (4, 1, 6),
          (8, 1, 0), (8, 1, 1), (8, 1, 2), (8, 1, 3), (8, 1, 4), (8, 1, 5), (8, 1, 6),
          (4, 0, 7), (4, 1, 7)]
INT64_MAX = "INT64_MAX"


def log(msg):
    print("[tune] " + msg, file=sys.stderr, flush=True)


def time_graph(calls, reps=7):
    """Median seconds per call of a graph running calls() once."""
    s = torch.cuda.Stream()
    calls()  # eager once (checks the arguments, warms the caches of code)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ncalls = calls()
    g.replay()
    torch.cuda.synchronize()
    out = []
    st = torch.cuda.current_stream()
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        g.replay()
        e1.record(st)
        e1.synchronize()
        out.append(e0.elapsed_time(e1) * 1e-3 / ncalls)
    del g
    return statistics.median(out)


def spills(bt, u, is_dot):
    """Launch shapes whose kernel instance spills registers: eight-vector
    dots in the instance built for blocks of more than 512 threads (128
    VGPRs). The table never picks them."""
    return bool(is_dot) and u == 8 and bt > 512


def single_candidates(quick, is_dot=0):
    bts = (256, 512) if quick else (256, 512, 1024)
    us = (2, 4, 8) if quick else (1, 2, 4, 8)
    gbs = (256, 512) if quick else (128, 256, 512, 1024, 2048)
    return [c for c in itertools.product(bts, us, gbs) if not spills(c[0], c[1], is_dot)]


def tune_single(dev, quick, combos, only_buckets=None, passes=1):
    rows = []
    # bucket upper bounds and the size timed for each
    buckets = [(1 << 14, 1 << 14), (1 << 18, 1 << 18), (1 << 22, 1 << 22), (1 << 24, 1 << 24),
               (1 << 25, 1 << 25), (INT64_MAX, None)]
    if only_buckets:
        buckets = [b for b in buckets if b[0] in only_buckets]
    big = {4: 1 << 28, 8: 1 << 27}  # 1 GiB per vector
    for dtype, is_dot, mode in combos:
        tdt = torch.float32 if dtype == 4 else torch.float64
        for n_max, n in buckets:
            n = n or big[dtype]
            per_call = n * dtype * (2 if is_dot else 1)
            # rotate over >= 1 GiB of distinct data (four times the last-level
            # cache) unless one call's inputs already exceed it
            copies = max(1, min(8, (1 << 30) // per_call))
            xs = [torch.empty(n, dtype=tdt, device=dev).uniform_(-1, 1) for _ in range(copies)]
            ys = [torch.empty(n, dtype=tdt, device=dev).uniform_(-1, 1) for _ in range(copies)] \
                if is_dot else [None] * copies
            reps = max(copies, min(64, (1 << 30) // (n * dtype)))
            outs = torch.empty((reps, 2), dtype=torch.float64, device=dev)
            def time_candidate(bt, u, gb):
                lc = tf.Launch(bt, u, gb, 0, 0)
                need = tf._lib.load().twofold_workspace_bytes_single(dtype, is_dot, mode, n, lc)
                ws = tf.Workspace(need, dev)

                def calls():
                    for r in range(reps):
                        x, y = xs[r % copies], ys[r % copies]
                        o = outs[r] if (dtype == 8 or mode in (3, 7)) else outs[r].view(torch.float32)[:2]
                        if mode == 3:
                            (tf.dotd(x, y, lc, out=o, ws=ws) if is_dot else tf.sumd(x, lc, out=o, ws=ws))
                        elif mode == 7:
                            (tf.dot_mixed(x, y, lc, out=o, ws=ws) if is_dot
                             else tf.sum_mixed(x, lc, out=o, ws=ws))
                        elif is_dot:
                            tf.dot(x, y, MODES[mode], lc, out=o, ws=ws)
                        else:
                            tf.sum(x, MODES[mode], lc, out=o, ws=ws)
                    return reps

                return time_graph(calls)

            # every pass times all candidates, in alternating order; a
            # candidate keeps its best time, so one slow replay does not
            # decide
            cands = single_candidates(quick, is_dot)
            times = {}
            for p in range(passes):
                for c in (cands if p % 2 == 0 else cands[::-1]):
                    t = time_candidate(*c)
                    times[c] = min(t, times.get(c, t))
            best = min((t,) + c for c, t in times.items())
            t, bt, u, gb = best
            gbs = n * dtype * (2 if is_dot else 1) / t / 1e9
            log("single dtype=%d dot=%d %s n=%d: bt=%d u=%d max_blocks=%d  %.2f us  %.0f GB/s"
                % (dtype, is_dot, MODES[mode], n, bt, u, gb, t * 1e6, gbs))
            rows.append("{0, %d, %d, %d, %s, INT64_MAX, %d, %d, %d, 0},  // %.0f GB/s at n=%d"
                        % (dtype, is_dot, mode, n_max, bt, u, gb, gbs, n))
            del xs, ys
            torch.cuda.empty_cache()
    return rows


# Mean segment length up to which the short-segment rows apply.
SHORT_LEN = 1024


def seg_candidates(quick, short):
    """(tile multiple tm, unroll, block threads, grid blocks). Short segments
    (each one tile, latency-bound) want many waves and little unroll; the
    tile size matters only for their rare long segments."""
    if short:
        if quick:
            return itertools.product((16,), (1, 2), (256,), (1024, 2048))
        return itertools.product((16, 64), (1, 2, 4), (256, 512), (512, 1024, 2048))
    return itertools.product((16, 64) if quick else (16, 32, 64, 128, 256, 512),
                             (2, 4) if quick else (2, 4, 8),
                             (256, 512) if quick else (256, 512, 1024),
                             (256, 1024) if quick else (256, 512, 1024))


def tune_seg(dev, quick, combos):
    import synth
    rows = []
    # (n_max, len_max, lengths): the short-segment rows come first, so that
    # they win for any total size when the mean length is at most SHORT_LEN
    buckets = [(INT64_MAX, SHORT_LEN, synth.segment_lengths(5, 500000, max_len=1 << 11)),
               ((1 << 24), INT64_MAX, synth.segment_lengths(3, 2000, max_len=1 << 14)),
               ((1 << 29), INT64_MAX, synth.segment_lengths(3, 20000, max_len=1 << 17)),
               (INT64_MAX, INT64_MAX, synth.segment_lengths(3, 20000, max_len=1 << 20))]
    if quick:
        buckets = buckets[:3]
    for dtype, is_dot, mode in combos:
        tdt = torch.float32 if dtype == 4 else torch.float64
        W = 16 // dtype
        for n_max, len_max, lengths in buckets:
            off = synth.offsets_from_lengths(lengths)
            n = int(off[-1])
            x = torch.empty(n, dtype=tdt, device=dev).uniform_(-1, 1)
            y = torch.empty(n, dtype=tdt, device=dev).uniform_(-1, 1) if is_dot else None
            best = None
            for tm, u, bt, gb in seg_candidates(quick, len_max != INT64_MAX):
                if spills(bt, u, is_dot):
                    continue
                lc = tf.Launch(bt, u, gb, 0, 64 * W * tm)
                plan = tf.SegPlan(off, tdt, is_dot, MODES[mode], lc)
                out = torch.empty((plan.nseg, 2), dtype=plan.out_dtype, device=dev)
                ws = tf.Workspace(plan.workspace_bytes, dev)

                def calls():
                    plan.execute(x, y, out=out, ws=ws)
                    return 1

                t = time_graph(calls)
                plan.close()
                if best is None or t < best[0]:
                    best = (t, bt, u, gb, 64 * W * tm)
            t, bt, u, gb, ts = best
            gbs = n * dtype * (2 if is_dot else 1) / t / 1e9
            log("seg dtype=%d dot=%d %s n=%d nseg=%d: bt=%d u=%d grid=%d tile=%d  %.1f us  %.0f GB/s"
                % (dtype, is_dot, MODES[mode], n, len(lengths), bt, u, gb, ts, t * 1e6, gbs))
            rows.append("{1, %d, %d, %d, %s, %s, %d, %d, %d, %d},  // %.0f GB/s at n=%d, %d segments"
                        % (dtype, is_dot, mode, n_max, len_max, bt, u, gb, ts, gbs, n,
                           len(lengths)))
            del x, y
            torch.cuda.empty_cache()
    return rows


HEADER = """// Tuned launch table: {kind, dtype, is_dot, mode, n_max, len_max,
// block_threads, unroll, max_blocks, tile_elems}. kind 0 single vector, 1
// segmented. Rows are searched in order; the first row whose n_max is at
// least the call's n (segmented: total elements) and whose len_max is at
// least its mean segment length wins. Single-vector rows give the
// largest grid: a call uses the blocks one round needs, at most max_blocks.
// Written by paper_1401_0248_amd/tune.py on %s; the comments give the
// throughput measured for the row's timed size.
"""


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--quick", action="store_true", help="fewer candidates (smoke use)")
    ap.add_argument("--only", choices=("single", "seg"), default=None)
    ap.add_argument("--combo", action="append", default=None, metavar="DTYPE,IS_DOT,MODE",
                    help="tune only these combinations (repeatable), e.g. 8,1,3")
    ap.add_argument("--bucket", action="append", default=None, metavar="N_MAX",
                    help="single vector: tune only the size buckets with this upper bound "
                         "(repeatable; 'max' for the last one)")
    ap.add_argument("--passes", type=int, default=1,
                    help="single vector: time every candidate this many times, keep its best")
    args = ap.parse_args()
    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    name = "a %s GPU" % getattr(props, "gcnArchName", props.name)
    t0 = time.time()
    combos = COMBOS
    if args.combo:
        combos = [tuple(int(v) for v in c.split(",")) for c in args.combo]
        for c in combos:
            if c not in COMBOS:
                ap.error("unknown combination %s" % (c,))
    rows = []
    if args.only in (None, "single"):
        only = None
        if args.bucket:
            only = [INT64_MAX if b == "max" else int(b) for b in args.bucket]
        rows += tune_single(dev, args.quick, combos, only, max(1, args.passes))
    if args.only in (None, "seg"):
        rows += tune_seg(dev, args.quick, combos)
    with open(args.out, "w") as f:
        f.write(HEADER % name)
        for r in rows:
            f.write(r + "\n")
    log("wrote %d rows to %s in %.0f s" % (len(rows), args.out, time.time() - t0))


if __name__ == "__main__":
    main()
