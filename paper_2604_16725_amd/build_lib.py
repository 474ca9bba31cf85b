"""Build the HIP library ``libflix.so`` for gfx950 in-tree.

    python -m paper_2604_16725_amd.build_lib

The library is four objects compiled in parallel (the C ABI with the sort,
update and partition kernels; the read kernels for 32-bit and for 64-bit keys;
the persistent drain) and linked into one shared object.  Every kernel is compiled for
gfx950 only, without packed-FP32 instructions.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
# (source, object, extra flags)
UNITS = [("flix.hip", "flix.o", []),
         ("flix_read_tu.hip", "flix_read32.o", ["-DFLIX_READ_KEY_BITS=32"]),
         ("flix_read_tu.hip", "flix_read64.o", ["-DFLIX_READ_KEY_BITS=64"]),
         ("flix_drain_tu.hip", "flix_drain_tu.o", [])]
SOURCES = sorted({u[0] for u in UNITS})
SRC = os.path.join(CSRC, SOURCES[0])
OUT_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(OUT_DIR, "libflix.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def build(verbose: bool = False) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    objs, procs = [], []
    for src, o, extra in UNITS:
        obj = os.path.join(OUT_DIR, o)
        cmd = ["hipcc", *HIPCC_FLAGS, *extra, "-c", "-o", obj + ".tmp", os.path.join(CSRC, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((subprocess.Popen(cmd), obj))
        objs.append(obj)
    failed = False
    for p, obj in procs:
        if p.wait() != 0:
            failed = True
        else:
            os.replace(obj + ".tmp", obj)
    if failed:
        raise subprocess.CalledProcessError(1, "hipcc (one of the translation units)")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-q" not in sys.argv))
