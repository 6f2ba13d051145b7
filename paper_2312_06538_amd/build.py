"""Compile the CRSH HIP library (libcrsh.so) for gfx950, in-tree.

Flags that the bit-exact contract depends on: no contraction into fused
multiply-add, correctly rounded float32 division and square root, denormals
kept.  Packed float32 instructions are disabled.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libcrsh.so")
SOURCES = ["api.hip", "hash.hip", "sort.hip", "build.hip", "traverse.hip", "hit.hip", "adjoint.hip", "batch.hip", "leafhit.hip", "sortchunk.hip"]
ARCH = os.environ.get("CRSH_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "-shared",
    f"--offload-arch={ARCH}",
    "-ffp-contract=off", "-fno-fast-math",
    "-fhip-fp32-correctly-rounded-divide-sqrt",
    "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose=False, out=None, defines=()):
    """Compile libcrsh.so (or `out`), with extra -D definitions if given."""
    lib = out or LIB
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    cmd = [hipcc(), *FLAGS, *[f"-D{d}" for d in defines], "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-o", lib + ".tmp", *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(lib + ".tmp", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
