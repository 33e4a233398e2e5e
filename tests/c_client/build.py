"""Build tests/c_client/client: a native C-ABI client of libtwofold.so,
linked against the in-tree library (rpath to the package directory)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
BIN = os.path.join(HERE, "client")


def build():
    pkg = os.path.join(ROOT, "paper_1401_0248_amd")
    cmd = [os.environ.get("HIPCC", "/opt/rocm/bin/hipcc"), "-O2", "-std=c++17",
           "-I" + os.path.join(ROOT, "include"), os.path.join(HERE, "client.cpp"),
           "-L" + pkg, "-ltwofold", "-Wl,-rpath,$ORIGIN/../../paper_1401_0248_amd",
           "-o", BIN + ".tmp"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("client build failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build())
