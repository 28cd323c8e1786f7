"""Build the gfx950 HIP library ``liblbm.so`` in-tree with hipcc.

Every call compiles from source.  Flags: gfx950 only, -O3, and packed-FP32
instructions disabled (-packed-fp32-ops) for all device code.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["kernels.hip", "abi.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=on: multiply-adds are fused only inside one source
# expression, as written, so every template instantiation of the collision
# (wall kinds, split or fused bounce-back, cells per lane) rounds identically;
# the default cross-statement fusion pairs products differently per kernel.
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=on",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-fvisibility=hidden", "-Wall", "-Wno-unused-result",
    "-I" + os.path.join(ROOT, "include"),
]


def build(verbose: bool = False, extra=()) -> str:
    cmd = [HIPCC] + FLAGS + list(extra) + [os.path.join(CSRC, s) for s in SOURCES] + \
        ["-o", LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
