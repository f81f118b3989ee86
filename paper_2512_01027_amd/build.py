"""Build step of the HIP library: compiles csrc/pulbm.hip into libpulbm.so
for gfx950 (MI355X) with hipcc.  Packed-FP32 instructions are disabled for
all device code."""
from __future__ import annotations

import os
import subprocess
import sys

_HERE = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_HERE)
LIB = os.path.join(_HERE, "libpulbm.so")


def build(verbose: bool = False, extra=()) -> str:
    src = os.path.join(_HERE, "csrc", "pulbm.hip")
    tmp = LIB + ".tmp"
    cmd = ["hipcc", "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wall", "-Wno-unused-function",
           "-I", os.path.join(_ROOT, "include"), "-I", os.path.join(_HERE, "csrc"),
           "-o", tmp, src, *extra]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
