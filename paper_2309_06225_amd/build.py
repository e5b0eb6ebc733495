"""Build libgrf.so in-tree: regenerate the pointwise device code, compile each
translation unit for gfx950 with hipcc (in parallel), link the shared library."""
from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "libgrf.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=fast-honor-pragmas",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]

# (source, object name, extra defines)
UNITS = [("libgrf.hip", "api", []), ("tu_stencil.hip", "stencil", []), ("tu_vjp.hip", "vjp", []),
         ("tu_vjp.hip", "vjp_dec", ["-DGRF_VJP_DEC=1"]),
         ("tu_constraints.hip", "constraints", []), ("tu_bc.hip", "bc", [])]
UNITS += [("tu_point.hip", f"point_m{m}", [f"-DGRF_TU_MODE={m}"]) for m in (0, 1, 2, 4)]
UNITS += [("tu_batch.hip", f"batch_m{m}", [f"-DGRF_TU_MODE={m}"]) for m in (1, 2, 4)]
UNITS += [("tu_staged.hip", f"staged_m{m}", [f"-DGRF_TU_MODE={m}"]) for m in (0, 1, 2, 4)]


def hipcc() -> str:
    for c in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def generate() -> dict:
    from .codegen import generate as G
    return G.main(os.path.join(CSRC, "gen"))


def _compile(unit, extra, verbose):
    src, name, defs = unit
    obj = os.path.join(OBJ, name + ".o")
    cmd = [hipcc()] + HIPCC_FLAGS + list(extra) + defs + ["-c", "-o", obj, os.path.join(CSRC, src)]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    return obj, r


def build(verbose: bool = False, extra=(), jobs: int | None = None) -> str:
    info = generate()
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or max(1, min(len(UNITS), os.cpu_count() or 1, 16))
    objs, failed = [], []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, r in ex.map(lambda u: _compile(u, extra, verbose), UNITS):
            objs.append(obj)
            if r.returncode != 0:
                failed.append((obj, r.stdout + r.stderr))
    if failed:
        for obj, log in failed:
            sys.stderr.write(f"--- {obj}\n{log}\n")
        raise RuntimeError("hipcc failed")
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", LIB + ".tmp"] + objs
    r = subprocess.run(cmd, cwd=CSRC, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(LIB + ".tmp", LIB)
    if verbose:
        print("built", LIB, info, flush=True)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
