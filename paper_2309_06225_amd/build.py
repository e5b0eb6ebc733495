"""Build libgrf.so in-tree: regenerate the pointwise device code, then hipcc for gfx950."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgrf.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=fast-honor-pragmas",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def generate() -> dict:
    from .codegen import generate as G
    return G.main(os.path.join(CSRC, "gen"))


def build(verbose: bool = False, extra=()) -> str:
    info = generate()
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra) + ["-o", LIB + ".tmp", os.path.join(CSRC, "libgrf.hip")]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB, info, flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
