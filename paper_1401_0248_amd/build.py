"""Build libtwofold.so (gfx950) in the package directory with hipcc.

Flags: strict IEEE (no FP contraction other than the explicit FMA, no
fast-math, binary32 subnormals kept) and no packed-FP32 instructions.

build_host_sanitized() builds the same library with AddressSanitizer and
UndefinedBehaviorSanitizer on its host code only (the argument checks, plan
creation, launch resolution), for the CPU sanitizer test; device code is
built as usual.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libtwofold.so")
SAN_DIR = os.path.join(HERE, "_build_san")
SAN_LIB = os.path.join(SAN_DIR, "libtwofold_san.so")
SOURCES = ["twofold.hip", "segmented.hip", "monitor.hip", "probes.hip", "batch.hip"]
DEPS = SOURCES + ["eft.hpp", "kernels.hpp", "host_common.hpp", "tuned_table.inc"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]
# host code only: each sanitizer flag goes to the host compilation alone
HOST_SANITIZE = [
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer",
    "-Xarch_host", "-g",
]
HOST_SANITIZE_LINK = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _newer(lib):
    if not os.path.exists(lib):
        return True
    t = os.path.getmtime(lib)
    deps = [os.path.join(CSRC, f) for f in DEPS] + [os.path.join(INCLUDE, "twofold.h")]
    return any(os.path.getmtime(p) > t for p in deps if os.path.exists(p))


def needs_build():
    return _newer(LIB)


def _compile_link(objdir, lib, extra, extra_link, quiet):
    """Compile every source into objdir in parallel, then link lib
    (replaced atomically)."""
    os.makedirs(objdir, exist_ok=True)
    procs = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        objs.append(obj)
        cmd = [HIPCC] + [f for f in FLAGS if f != "-shared"] + extra + [
            "-I" + INCLUDE, "-I" + CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((cmd, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE,
                                            text=True)))
    for cmd, p in procs:
        out, err = p.communicate()
        if p.returncode != 0:
            raise RuntimeError("hipcc failed:\n%s\n%s%s" % (" ".join(cmd), out, err))
        if not quiet and err:
            sys.stderr.write(err)
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + extra_link + ["-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, lib)
    return lib


def build(force=False, quiet=True):
    """Compile every source into libtwofold.so."""
    if not force and not needs_build():
        return LIB
    return _compile_link(os.path.join(HERE, "_build"), LIB, [], [], quiet)


def build_host_sanitized(force=False, quiet=True):
    """The library with sanitized host code, in _build_san/ (rebuilt only
    when a source changed). Loading it needs the compiler's AddressSanitizer
    runtime preloaded (clang_asan_runtime())."""
    if not force and not _newer(SAN_LIB):
        return SAN_LIB
    return _compile_link(SAN_DIR, SAN_LIB, HOST_SANITIZE, HOST_SANITIZE_LINK, quiet)


def clang_asan_runtime():
    """The AddressSanitizer runtime of hipcc's clang (shared)."""
    r = subprocess.run([HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"],
                       capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path):
        return path
    import glob
    found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return found[0] if found else None


if __name__ == "__main__":
    print(build(force=True, quiet=False))
