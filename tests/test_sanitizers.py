"""CPU runs under AddressSanitizer and UndefinedBehaviorSanitizer.

* The oracle (liboracle: the exact accumulator's digit indexing, the
  sequential loops, the order model's allocations) and the input
  generator's C helper (libsynth) are built with gcc's sanitizers, and the
  oracle's pin tests run against those builds in a fresh interpreter with
  gcc's ASan runtime preloaded (the TWOFOLD_ORACLE_LIB and
  TWOFOLD_SYNTH_LIB hooks).
* The HIP library is built with sanitized host code (argument checks, plan
  tables, launch resolution; device code as usual) and the C interface's
  CPU tests run against it with clang's ASan runtime preloaded (the
  TWOFOLD_HIP_LIB hook).

Any report aborts the run (halt_on_error, no recovery), so a clean exit is a
clean run. Leak detection is off: the interpreter keeps its allocations.
"""
import os
import subprocess
import sys

import pytest

from oracle import build as obuild
from paper_1401_0248_amd import build as hbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g"]
ENV = {"ASAN_OPTIONS": "detect_leaks=0:abort_on_error=1:alloc_dealloc_mismatch=0",
       "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"}
ORACLE_PINS = ["tests/test_xacc.py", "tests/test_oracle_eft.py", "tests/test_oracle_paper.py",
               "tests/test_model.py", "tests/test_mixed.py", "tests/test_model_order.py",
               "tests/test_bounds.py", "tests/test_monitor.py", "tests/test_generators.py"]


def _gcc_asan():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def _run(files, env, extra=()):
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu",
                        "-p", "no:cacheprovider"] + list(extra) + files,
                       cwd=ROOT, env=dict(os.environ, **ENV, **env), capture_output=True,
                       text=True, timeout=1200)
    return r.returncode, (r.stdout + r.stderr)[-3000:]


def test_oracle_and_generator_under_sanitizers(tmp_path):
    asan = _gcc_asan()
    if asan is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    flags = [f for f in obuild.CFLAGS if f != "-O2"] + ["-O1"] + SAN
    lib = str(tmp_path / "liboracle_san.so")
    r = subprocess.run(["gcc"] + flags + ["-o", lib] +
                       [os.path.join(obuild.HERE, s) for s in obuild.SOURCES] + ["-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    synth_lib = str(tmp_path / "libsynth_san.so")
    r = subprocess.run(["gcc", "-O1", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math"] +
                       SAN + ["-o", synth_lib, os.path.join(ROOT, "synth", "illcond.c"), "-lm"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    # the 2^24-element generator pin is left to the plain run (time only)
    rc, tail = _run(ORACLE_PINS, {"LD_PRELOAD": asan, "TWOFOLD_ORACLE_LIB": lib,
                                  "TWOFOLD_SYNTH_LIB": synth_lib},
                    ["-k", "not reaches_its_decade"])
    assert rc == 0, tail


def test_host_checks_under_sanitizers():
    asan = hbuild.clang_asan_runtime()
    if asan is None:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    lib = hbuild.build_host_sanitized()
    rc, tail = _run(["tests/test_api_cpu.py"], {"LD_PRELOAD": asan, "TWOFOLD_HIP_LIB": lib})
    assert rc == 0, tail
