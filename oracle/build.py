"""Build the oracle's shared library with gcc (strict IEEE: no contraction,
no fast-math, SSE2 arithmetic). Test infrastructure only."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = ["xacc.c", "paper_loops.c", "order_model.c"]
DEPS = SOURCES + ["paper_loops.inc", "order_model.inc", "twofold_oracle.h", "dw.h"]
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = [
    "-O2", "-std=gnu11", "-fPIC", "-shared", "-pthread",
    "-ffp-contract=off", "-fno-fast-math", "-msse2", "-mfpmath=sse",
    "-fno-strict-aliasing", "-Wall", "-Wextra", "-Wno-unused-parameter",
]


def needs_build():
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(os.path.join(HERE, f)) > t for f in DEPS)


def build(force=False, quiet=True):
    if not force and not needs_build():
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc"] + CFLAGS + ["-o", tmp] + [os.path.join(HERE, s) for s in SOURCES] + ["-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("oracle build failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    if not quiet and r.stderr:
        sys.stderr.write(r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(force=True, quiet=False))
