"""Build libgsf.so in-tree with hipcc for gfx950.

The library is the C ABI of include/gsf.h: host dispatch (gsf_api.cpp,
gsf_prof.cpp) plus the HIP kernels (gsf_kernels.hip, gsf_filter.hip,
gsf_stats.hip, and the merged spatial sweeps of gsf_merged.h instantiated
per storage type in gsf_merged_*.hip).  Packed FP32 instructions are disabled for every device
function (-packed-fp32-ops).  Objects go to _build/ (not tracked).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgsf.so")
SOURCES = ["gsf_api.cpp", "gsf_prof.cpp", "gsf_kernels.hip", "gsf_filter.hip", "gsf_stats.hip",
           "gsf_merged_f32.hip", "gsf_merged_f16.hip", "gsf_merged_bf16.hip"]
ARCH = "gfx950"


FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-Wall",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
OBJDIR = os.path.join(HERE, "_build")


def hipcc_cmd(out: str, extra: list[str] | None = None) -> list[str]:
    """One hipcc invocation that compiles and links every source."""
    return (["/opt/rocm/bin/hipcc"] + FLAGS + ["-shared"] + (extra or []) + ["-o", out, "-x", "hip"]
            + [os.path.join(CSRC, s) for s in SOURCES])


def build(verbose: bool = False, extra: list[str] | None = None, out: str = LIB) -> str:
    """Compile the sources to objects in parallel (one hipcc per file), then
    link libgsf.so; the library is replaced only once the link succeeds."""
    from concurrent.futures import ThreadPoolExecutor

    os.makedirs(OBJDIR, exist_ok=True)
    objs = [os.path.join(OBJDIR, os.path.splitext(s)[0] + ".o") for s in SOURCES]
    cmds = [["/opt/rocm/bin/hipcc"] + FLAGS + (extra or []) + ["-c", "-o", o, "-x", "hip",
                                                               os.path.join(CSRC, s)]
            for s, o in zip(SOURCES, objs)]
    workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        results = list(pool.map(lambda c: subprocess.run(c, capture_output=True, text=True), cmds))
    for c, r in zip(cmds, results):
        if verbose:
            print(" ".join(c), flush=True)
        if r.stderr and (verbose or r.returncode):
            print(r.stderr, end="", file=sys.stderr, flush=True)
        if r.returncode:
            raise subprocess.CalledProcessError(r.returncode, c)
    tmp = out + ".tmp"
    link = ["/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(link), flush=True)
    subprocess.run(link, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
