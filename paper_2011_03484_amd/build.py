"""Build ``libtpmvs.so`` (HIP kernels + host runtime + C ABI) for gfx950 in-tree."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libtpmvs.so")
SOURCES = ["kernels_core.hip", "ad_kernels.hip", "diag_kernels.hip", "history.hip",
           "handoff.hip", "runtime.hip", "static_run.hip"]
HEADERS = ["dmath.hpp", "kepler.hpp", "particle.hpp", "universal.hpp", "ad.hpp", "internal.h",
           "ad_internal.h", "diag_internal.h", "history_internal.h"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # explicit fma() everywhere; no compiler contraction, no fast-math
    "-ffp-contract=off",
    # never emit packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # FP64 FMAs as three-address v_fma_f64: the two-address v_fmac_f64
    # overwrites its addend, so an addend that stays live (a series constant
    # held in a VGPR, a value used again) costs a v_mov_b64 copy per FMA (the
    # planet-map kernels turn it back on for themselves)
    "-Xclang", "-target-feature", "-Xclang", "-fmacf64-inst",
    "-Wno-unused-result",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link the shared library (always rebuilds)."""
    objs = []
    for src in sources():
        obj = os.path.join(CSRC, os.path.basename(src) + ".o")
        cmd = [HIPCC, *FLAGS, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
