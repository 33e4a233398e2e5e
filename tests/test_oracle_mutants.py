"""Planted mistakes in the oracle, caught on the CPU by its pins.

Each mutant is a copy of the oracle's C sources with one plausible slip (a
dropped term, a wrong sign, a swapped or wrong operand), compiled with the
oracle's own flags into a library of its own. The oracle's pin tests then
run in a fresh interpreter against that library (the conftest hook
TWOFOLD_ORACLE_LIB points the oracle at it) and must fail. The unchanged
copy, built the same way, must pass them, so a failure is the slip's and
not the harness's.

The slips cover the three parts of the oracle: the exact accumulator, the
paper's sequential loops and the order model (steps, combines, grid
combine, finalize, the mixed and double-word forms, and the order itself).
Slips that only reorder a reduction (a lane or chain index, the width of a
combine) leave every value that the mathematics fixes exact or within its
bound; the numpy statement of the order (tests/test_model_order.py)
catches those.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import build as obuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_xacc.py", "tests/test_oracle_eft.py", "tests/test_oracle_paper.py",
             "tests/test_model.py", "tests/test_mixed.py", "tests/test_model_order.py"]

# (name, file, text, replacement): the text occurs exactly once in the file
MUTANTS = [
    # exact accumulator
    ("xacc product sign", "xacc.c", "absval ? 0 : (nx ^ ny))", "absval ? 0 : (nx | ny))"),
    ("xacc exponent off by one", "xacc.c", "*e = ex - 53;", "*e = ex - 52;"),
    ("xacc carry sign", "xacc.c", "a->dig[i + 1] += c;", "a->dig[i + 1] -= c;"),
    # the paper's sequential methods
    ("fast-two-sum remainder sign", "paper_loops.inc",
     "  *r = b - (t - a);", "  *r = (t - a) - b;"),
    ("two-sum dropped the first operand's part", "paper_loops.inc",
     "  *r = (a - av) + (b - bv);", "  *r = (b - bv);"),
    ("two-sum second part sign", "paper_loops.inc",
     "  *r = (a - av) + (b - bv);", "  *r = (a - av) + (bv - b);"),
    ("two-sum first part operand", "paper_loops.inc",
     "  const T av = t - bv;", "  const T av = t - b;"),
    ("Kahan correction sign", "paper_loops.inc",
     "NAME(fts)(s, item + k, &s, &k);", "NAME(fts)(s, item - k, &s, &k);"),
    ("twofold dot dropped product remainder", "paper_loops.inc",
     "if (y && exact_product) r = r + FMA(x[i], y[i], -item);",
     "if (y && exact_product) r = r;"),
    ("twofold dot product remainder sign", "paper_loops.inc",
     "if (y && exact_product) r = r + FMA(x[i], y[i], -item);",
     "if (y && exact_product) r = r - FMA(x[i], y[i], -item);"),
    ("twofold error sign", "paper_loops.inc", "    e = e + r;", "    e = e - r;"),
    ("dot swapped factor", "paper_loops.inc",
     "  for (int64_t i = 0; i < n; i++) s = s + x[i] * y[i];",
     "  for (int64_t i = 0; i < n; i++) s = s + x[i] * x[i];"),
    # order model: steps
    ("model two-sum second part sign", "order_model.inc",
     "  *r = (a - av) + (b - bv);", "  *r = (a - av) + (bv - b);"),
    ("model two-sum first part operand", "order_model.inc",
     "  A av = t - bv;", "  A av = t - b;"),
    ("model fast-two-sum remainder sign", "order_model.inc",
     "  *r = b - (t - a);", "  *r = (t - a) - b;"),
    ("model dot dropped product remainder", "order_model.inc",
     "if (track) r = r + (A)FMA_T(xv, yv, -p);", "if (track) r = r;"),
    ("model dot product remainder sign", "order_model.inc",
     "if (track) r = r + (A)FMA_T(xv, yv, -p);", "if (track) r = r - (A)FMA_T(xv, yv, -p);"),
    ("model Kahan sign", "order_model.inc",
     "NAME(fts)(*s, item + *e, s, e);", "NAME(fts)(*s, item - *e, s, e);"),
    # order model: combines, grid combine, finalize
    ("combine dropped partner error", "order_model.inc",
     "  *e1 = (*e1 + e2) + y;\n  *s1 = x;", "  *e1 = *e1 + y;\n  *s1 = x;"),
    ("combine two-sum sign", "order_model.inc", "  A bh = b - bp;", "  A bh = bp - b;"),
    ("grid combine dropped remainder", "order_model.c",
     "  double y = ah + bh;\n  *e1 = (*e1 + e2) + y;", "  double y = ah + bh;\n  *e1 = *e1 + e2;"),
    ("binary32 finalize dropped rest", "order_model.c", "e = (float)(rest + E);", "e = (float)E;"),
    ("wide chains not widened", "order_model.inc",
     "A item = is_dot ? (A)xv * (A)yv : (A)xv;", "A item = is_dot ? (A)(xv * yv) : (A)xv;"),
    # the mixed form
    ("mixed dot dropped remainder", "order_model.inc",
     "*e = *e + ((double)r + (double)fmaf(xf, yf, -p));", "*e = *e + (double)r;"),
    ("mixed error kept in binary32", "order_model.inc",
     "      *e = *e + (double)r;\n    *s = (A)t;",
     "      *e = (float)(*e + (double)r);\n    *s = (A)t;"),
    ("mixed two-sum sign", "order_model.c",
     "  *r = (a - av) + (b - bv);", "  *r = (a - av) - (b - bv);"),
    ("mixed finalize error narrowed", "order_model.c",
     "out2[1] = (V - v) + E;", "out2[1] = (double)(float)((V - v) + E);"),
    # order model: the order itself
    ("order: rounds contiguous per lane", "order_model.inc",
     "int64_t k = q * per_round + (int64_t)u * L + g;", "int64_t k = q * per_round + g * U + u;"),
    ("order: head elements on one lane's chains", "order_model.inc",
     "    NAME(step)(mode, is_dot, &cs[i * W], &ce[i * W], x[el], is_dot ? y[el] : (T)0, viol);\n"
     "  }\n  int64_t per_round",
     "    NAME(step)(mode, is_dot, &cs[i], &ce[i], x[el], is_dot ? y[el] : (T)0, viol);\n"
     "  }\n  int64_t per_round"),
    ("order: 128 grid-combine lanes", "order_model.inc",
     "grid_combine64(mode, qs, qe, GB, 256, &V, &E);", "grid_combine64(mode, qs, qe, GB, 128, &V, &E);"),
    ("order: 128 tile-combine lanes", "order_model.inc",
     "grid_combine64(mode, ts, te, ntiles, 64, &V, &E);",
     "grid_combine64(mode, ts, te, ntiles, 128, &V, &E);"),
    ("order: butterflies reversed", "order_model.c",
     "  for (int d = 1; d < 64; d <<= 1) {\n    for (int l = 0; l < 64; l++) {\n      ns[l] = s[l];",
     "  for (int d = 32; d >= 1; d >>= 1) {\n    for (int l = 0; l < 64; l++) {\n      ns[l] = s[l];"),
    # double-word additions
    ("double-word dropped low sum", "dw.h", "  double c = sl + th;", "  double c = sl;"),
    ("double-word two-sum sign", "dw.h", "*d = (a - av) + (b - bv);", "*d = (a - av) - (b - bv);"),
]


# Slips in the error bounds (oracle/bounds.py), run against the bound pins
# (the bound tests pin each bound from below and from above).
BOUND_PIN_FILES = ["tests/test_bounds.py", "tests/test_model.py", "tests/test_mixed.py"]
BOUND_MUTANTS = [
    ("double-word bound: u for u^2", "3 * u * u + 13 * u ** 3", "3 * u + 13 * u ** 3"),
    ("fast loss term dropped", "loss = u * (1 + 2 * u) * fast_violations",
     "loss = 0.0 * fast_violations"),
    ("fast loss term: u^2 for u", "loss = u * (1 + 2 * u) * fast_violations",
     "loss = u * u * fast_violations"),
    ("tree bound: factor u dropped from the terms", "T = u * (Lc + D + 1) * grow * A + loss",
     "T = (Lc + D + 1) * grow * A + loss"),
    ("tree bound 10^4 too tight", "b = g(h, u) * T + loss", "b = 1e-4 * g(h, u) * T + loss"),
    ("mixed bound: binary32 rounding for the binary64 error sum", "return g(h, u64) * T + u64 *",
     "return g(h, u32) * T + u64 *"),
]


def _bound_mutant(tmp, i, name, text, repl):
    src = open(os.path.join(ROOT, "oracle", "bounds.py")).read()
    assert src.count(text) == 1, (name, src.count(text))
    path = os.path.join(tmp, "bounds_m%02d.py" % i)
    with open(path, "w") as f:
        f.write(src.replace(text, repl))
    env = dict(os.environ, TWOFOLD_BOUNDS_PY=path, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider"] + BOUND_PIN_FILES,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, (r.stdout + r.stderr)[-1500:]


def _sources(dst):
    for f in obuild.DEPS:
        shutil.copy(os.path.join(obuild.HERE, f), os.path.join(dst, f))


def _compile(d, name):
    lib = os.path.join(d, "liboracle_%s.so" % name)
    cmd = ["gcc"] + obuild.CFLAGS + ["-o", lib] + [os.path.join(d, s) for s in obuild.SOURCES] + \
        ["-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return lib


def _pins(lib):
    """Run the pin tests against lib; returns pytest's exit status and the
    tail of its report."""
    env = dict(os.environ, TWOFOLD_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider"] + PIN_FILES,
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, (r.stdout + r.stderr)[-1500:]


def _mutant(tmp, i, name, fname, text, repl):
    d = os.path.join(tmp, "m%02d" % i)
    os.makedirs(d)
    _sources(d)
    path = os.path.join(d, fname)
    src = open(path).read()
    assert src.count(text) == 1, (name, src.count(text))
    with open(path, "w") as f:
        f.write(src.replace(text, repl))
    return _pins(_compile(d, "m%02d" % i))


@pytest.fixture(scope="module")
def tmp(tmp_path_factory):
    return str(tmp_path_factory.mktemp("oracle_mutants"))


def test_unchanged_copy_passes_the_pins(tmp):
    d = os.path.join(tmp, "clean")
    os.makedirs(d)
    _sources(d)
    rc, tail = _pins(_compile(d, "clean"))
    assert rc == 0, tail


def test_every_planted_mistake_fails_a_pin(tmp):
    with ThreadPoolExecutor(max_workers=4) as pool:
        futs = [pool.submit(_mutant, tmp, i, *m) for i, m in enumerate(MUTANTS)]
        results = [f.result() for f in futs]
    survivors = [(m[0], tail) for m, (rc, tail) in zip(MUTANTS, results) if rc != 1]
    assert not survivors, survivors


def test_unchanged_bounds_copy_passes_the_bound_pins(tmp):
    rc, tail = _bound_mutant(tmp, 99, "unchanged", "import math", "import math")
    assert rc == 0, tail


def test_every_planted_bound_mistake_fails_a_pin(tmp):
    with ThreadPoolExecutor(max_workers=4) as pool:
        futs = [pool.submit(_bound_mutant, tmp, i, *m) for i, m in enumerate(BOUND_MUTANTS)]
        results = [f.result() for f in futs]
    survivors = [(m[0], tail) for m, (rc, tail) in zip(BOUND_MUTANTS, results) if rc != 1]
    assert not survivors, survivors
