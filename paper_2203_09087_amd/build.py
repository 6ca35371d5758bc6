"""Builds the HIP library ``libecc_hip.so`` for gfx950 with hipcc (in-tree).

Compiles on any machine with ROCm (no GPU needed).  The flags keep the float
arithmetic of the binning step exact to the documented formula (no contraction)
and keep the compiler away from packed FP32 instructions.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libecc_hip.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("ecc_api.hip", "ecc_kernels.hip", "ecc_reduce.hip", "ecc_batch.hip", "ecc_smooth.hip")]

HIPCC_FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
    "-I", os.path.join(ROOT, "include"),
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", "hipcc"):
        if cand and (os.path.sep not in cand or os.path.exists(cand)):
            return cand
    return "hipcc"


def build(verbose: bool = False, out: str = LIB, defines=()) -> str:
    """Compiles every HIP source into `out` (always recompiles).

    defines: extra preprocessor definitions ("NAME=VALUE"), used for tuning builds."""
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *[f"-D{d}" for d in defines], *SOURCES, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
