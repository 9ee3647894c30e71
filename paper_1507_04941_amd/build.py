"""Build libgsf.so in-tree with hipcc for gfx950.

The library is the C ABI of include/gsf.h: host dispatch (gsf_api.cpp) plus
the HIP kernels (gsf_kernels.hip).  Packed FP32 instructions are disabled for
every device function (-packed-fp32-ops).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsf.so")
SOURCES = ["gsf_api.cpp", "gsf_prof.cpp", "gsf_kernels.hip", "gsf_filter.hip", "gsf_stats.hip"]
ARCH = "gfx950"


def hipcc_cmd(out: str, extra: list[str] | None = None) -> list[str]:
    return (["/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
             "-shared", "-Wall", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
            + (extra or []) + ["-o", out, "-x", "hip"] + [os.path.join(CSRC, s) for s in SOURCES])


def build(verbose: bool = False) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
