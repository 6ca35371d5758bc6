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
    """Compiles every HIP source into `out` (always recompiles): one object per
    source, compiled in parallel, then one shared library.  The sources share no
    device code, so no relocatable device code is needed.

    defines: extra preprocessor definitions ("NAME=VALUE"), used for tuning builds."""
    import tempfile
    from concurrent.futures import ThreadPoolExecutor
    compile_flags = [f for f in HIPCC_FLAGS if f != "-shared"]
    defs = [f"-D{d}" for d in defines]
    with tempfile.TemporaryDirectory(prefix="ecc_build_") as tmpdir:
        objs = [os.path.join(tmpdir, os.path.basename(src) + ".o") for src in SOURCES]
        cmds = [[hipcc(), *compile_flags, *defs, "-c", src, "-o", obj] for src, obj in zip(SOURCES, objs)]
        if verbose:
            for c in cmds:
                print(" ".join(c), flush=True)
        jobs = max(1, min(len(cmds), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(jobs) as ex:
            results = list(ex.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
        for c, r in zip(cmds, results):
            if r.returncode != 0:
                print(r.stderr, flush=True)
                raise subprocess.CalledProcessError(r.returncode, c, r.stdout, r.stderr)
        tmp = out + ".tmp"
        link = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
