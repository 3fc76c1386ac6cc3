"""Build the HIP library libcoreals.so for gfx950 (in-tree, next to this file).

Each source compiles to its own object in parallel (no device code crosses a
translation unit), then one link makes the shared library.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libcoreals.so")
SOURCES = ["capi.hip", "setup.hip", "sweep.hip", "heavy.hip", "wide.hip", "objective.hip", "foldin.hip",
           "fast.hip", "unif.hip", "implicit.hip",
           "noalloc.hip"]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    # no packed FP32 instructions anywhere in this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def sources() -> list:
    return [s for s in SOURCES if os.path.exists(os.path.join(SRC, s))]


def build(verbose: bool = False, jobs: int = 8) -> str:
    os.makedirs(OBJ, exist_ok=True)
    srcs = sources()

    def compile_one(s):
        obj = os.path.join(OBJ, s.replace(".hip", ".o"))
        cmd = [hipcc(), *HIPCC_FLAGS, "-c", "-o", obj, os.path.join(SRC, s)]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        # hipcc's host pass does not know the packed-FP32 feature: harmless
        msg = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed on {s}:\n{msg}")
        if verbose and msg.strip():
            print(msg, flush=True)
        return obj

    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(srcs)))) as ex:
        objs = list(ex.map(compile_one, srcs))
    tmp = LIB + ".tmp"
    subprocess.check_call([hipcc(), "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
