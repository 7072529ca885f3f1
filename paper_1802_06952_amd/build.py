"""Build libqs.so in-tree with hipcc for gfx950.

    python -m paper_1802_06952_amd.build        (or python paper_1802_06952_amd/build.py)

Compiles every source under csrc/ into one shared library next to this file.
Packed FP32 instructions are switched off for the device code, and MFMA
results are kept in ordinary vector registers.
"""

from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libqs.so")


def hipcc() -> str:
    for c in ("/opt/rocm/bin/hipcc", shutil.which("hipcc") or ""):
        if c and os.path.exists(c):
            return c
    raise RuntimeError("hipcc not found")


def build(verbose: bool = True, extra: list[str] | None = None) -> str:
    srcs = sorted(glob.glob(os.path.join(HERE, "csrc", "*.cpp")) +
                  glob.glob(os.path.join(HERE, "csrc", "*.hip")))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           # MFMA accumulators in ordinary VGPRs: without it the FP32 GEMM's
           # loop copies every accumulator between AGPRs and VGPRs
           "-mllvm", "-amdgpu-mfma-vgpr-form",
           "-I", os.path.join(os.path.dirname(HERE), "include"),
           *srcs, "-o", tmp] + (extra or [])
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed")
    if verbose and r.stderr.strip():
        # host pass warns about the device-only feature flag; keep other warnings visible
        lines = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln]
        if lines:
            sys.stderr.write("\n".join(lines) + "\n")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
