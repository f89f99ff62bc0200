"""Build libpufe.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpufe.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["capi.cpp", "plan.cpp", "kernels.hip", "backward.hip", "split.hip", "aq_error.hip", "nonlocal.hip",
           "bloch.hip", "scf.hip"]
HEADERS = ["tables.hpp", "plan.hpp", "kernels.hpp", "basis.hpp", "backward.hpp", "device_common.hpp", "enrich.hpp",
           "aq_error.hpp", "stage.hpp", "limbs.hpp", "nonlocal.hpp", "bloch.hpp", "scf.hpp"]

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC",
    # packed FP32 instructions stay off in every HIP build of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def _hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if c and (os.path.sep not in c or os.path.exists(c)):
            return c
    return "hipcc"


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source of the library (one object per source, in
    parallel) and link them; always rebuilds."""
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(HERE, "..", "include")]

    def compile_one(src):
        obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
        cmd = [_hipcc(), *FLAGS, *inc, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        return obj

    with ThreadPoolExecutor(max_workers=max(1, min(jobs, len(SOURCES)))) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    files = [os.path.join(CSRC, s) for s in SOURCES + HEADERS]
    files.append(os.path.join(HERE, "..", "include", "pufe.h"))
    return any(os.path.getmtime(f) > t for f in files if os.path.exists(f))


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
