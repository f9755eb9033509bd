"""Compile the HIP library for gfx950 into this package directory.

    python -m paper_1611_05319_amd.build

The library is built in-tree (libguidefill.so next to this file).  Flags:
FP64 geometry must not be contracted into FMA (-ffp-contract=off), packed
FP32 instructions are disabled, hardware float atomics are used for the
adjoint's scatter into device memory.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "guidefill.hip")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libguidefill.so")
ARCH = os.environ.get("GF_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def command(out: str) -> list[str]:
    return [hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
            "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function", f"-I{INCLUDE}", SRC,
            "-o", out]


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
    sys.exit(0)
