"""Build the HIP library (gfx950) in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgks.so")
SOURCES = [os.path.join(HERE, "csrc", "gks_device.hip"), os.path.join(HERE, "csrc", "gks_prep.cpp")]
DEPS = SOURCES + [os.path.join(HERE, "csrc", "gks_flux.h"), os.path.join(HERE, "csrc", "gks_internal.h"),
                  os.path.join(HERE, "csrc", "gks_flux_adj.h"), os.path.join(HERE, "csrc", "gks_opcount.h"),
                  os.path.join(HERE, "csrc", "gks_bc.h"), os.path.join(HERE, "csrc", "gks_weno.h"),
                  os.path.join(ROOT, "include", "gks.h")]

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared", "-fopenmp",
    # packed FP32 instructions stay off in every HIP build of this library
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    cmd = [hipcc(), *HIPCC_FLAGS, "-I" + os.path.join(ROOT, "include"), "-o", LIB + ".tmp", *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    build(verbose=True)
