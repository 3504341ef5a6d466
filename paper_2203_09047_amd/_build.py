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
# the kernels' source only: no loop-invariant hoisting after instruction selection.  In the flux
# kernels' loops over chunks it lifts dozens of FP64 constants and parameter-derived values out of
# the loop, each then held in registers (or spilled) across the whole flux evaluation.  (hipcc
# passes -mllvm options to the host compilation as well, so the host preprocessor is compiled apart.)
DEVICE_FLAGS = ["-mllvm", "-disable-machine-licm"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.isabs(cand) and os.path.exists(cand) or not os.path.isabs(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False) -> str:
    inc = "-I" + os.path.join(ROOT, "include")
    prep_o, dev_o = LIB + ".prep.o", LIB + ".dev.o"
    flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    steps = [
        [hipcc(), "-O3", "-std=c++17", "-fPIC", "-fopenmp", inc, "-c", "-o", prep_o, SOURCES[1]],
        [hipcc(), *flags, *DEVICE_FLAGS, inc, "-c", "-o", dev_o, SOURCES[0]],
        [hipcc(), *HIPCC_FLAGS, "-o", LIB + ".tmp", dev_o, prep_o],
    ]
    for cmd in steps:
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.remove(prep_o)
    os.remove(dev_o)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def stale() -> bool:
    if not os.path.exists(LIB):
        return True
    t = os.path.getmtime(LIB)
    return any(os.path.getmtime(d) > t for d in DEPS)


if __name__ == "__main__":
    build(verbose=True)
