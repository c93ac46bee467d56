"""Build libndgp.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_1511_08200_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libndgp.so")
SOURCES = ["ndgp_kernels.hip", "ndgp_mixed.hip", "ndgp_solver.hip", "ndgp_screening.hip", "ndgp_amr.hip",
           "ndgp_boxes.hip", "ndgp_stats.hip", "ndgp_particles.hip"]
ARCH = os.environ.get("NDGP_OFFLOAD_ARCH", "gfx950")
ROCM_LIB = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm)")


def build(verbose: bool = False) -> str:
    """Compile every HIP source of the library into one shared object."""
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
           # packed FP32 instructions are kept out of every kernel
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           # no implicit fused multiply-adds: the same expression rounds the same
           # way in every kernel it is inlined into (fma() is written out)
           "-ffp-contract=off",
           "-Wall", "-Wno-unused-function",
           "-I", INCLUDE, "-I", CSRC, "-o", tmp] + [os.path.join(CSRC, s) for s in SOURCES] + [
           # host ranges for rocprofv3 --marker-trace
           f"-L{ROCM_LIB}", f"-Wl,-rpath,{ROCM_LIB}", "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
