"""bench.py's oracle leg on the CPU (no GPU): the sequential oracle's timed
sample, the grading of every segment against the exact accumulator, the
accumulator's one-thread rate and the sampled bitwise parity, fed with the
order model's own outputs at a fixed launch. A planted error in one output
must show up in the parity count."""
import numpy as np
import pytest


def _state(torch, bench, oracle, synth, nseg=200):
    lengths = synth.segment_lengths(3, nseg, max_len=1 << 12)
    off = synth.offsets_from_lengths(lengths)
    n = int(off[-1])
    host = {"float64": synth.uniform_fill(3, 2 * n, np.float64),
            "float32": synth.uniform_fill(3, 2 * n, np.float32)}

    class Launch:
        unroll, tile_elems, block_threads, grid_blocks = 4, 1024, 256, 64

    class Plan:
        launch = Launch()

    execs = []
    for name, form in bench.SEG_FORMS:
        x, y = host[name][:n], host[name][n:]
        out = oracle.model_seg(form, x, off, y, x_misalign=0, unroll=4, tile_elems=1024)
        execs.append({"name": name, "form": form, "plan": Plan(),
                      "out": torch.from_numpy(np.asarray(out, dtype=np.float64))})
    return {"off": off, "n": n, "host": host, "execs": execs}


def test_seg_oracle_leg_on_model_outputs(monkeypatch):
    torch = pytest.importorskip("torch")
    import bench
    import oracle
    import synth
    monkeypatch.setattr(bench, "ORACLE_SAMPLE_S", 0.5)
    monkeypatch.setattr(bench, "XACC_SAMPLE_S", 0.2)
    state = _state(torch, bench, oracle, synth)
    base, acc, parity = bench.seg_oracle_leg(np, torch, state)
    assert parity["mismatches"] == 0 and parity["forms"] == len(bench.SEG_FORMS)
    assert base["kind"] == "oracle" and base["cores"] == 1 and base["value"] > 0
    assert acc["segments_graded"] == 200
    ex = acc["exact_accumulator"]
    assert ex["one_thread_gelem_s"] > 0 and ex["all_threads_gelem_s"] > 0 and ex["threads"] >= 1
    for name in ("float64", "float32"):
        r = acc["%s_rigorous" % name]
        assert r["segments_over_4Lu2_bound"] == 0
        assert 0 <= r["max_over_tree_bound"] <= 1.0

    # one wrong bit in one output of the longest segment: the parity count sees it
    lens = np.diff(state["off"])
    s = int(np.argmax(lens))
    o = state["execs"][0]["out"]
    o[s, 1] = float(np.nextafter(o[s, 1].item(), np.inf))
    _, _, parity2 = bench.seg_oracle_leg(np, torch, state)
    assert parity2["mismatches"] == 1
