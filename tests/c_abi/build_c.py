"""Build the plain C caller of libgsf (tests/c_abi/find_from_c.c) next to its
source: gcc, C99, the library's public header and the HIP runtime API only,
linked against libgsf.so and, as its checker, the oracle's shared library
(both found through rpaths relative to the binary)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "find_from_c.c")
BIN = os.path.join(HERE, "find_from_c")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", "/opt/rocm/include", SRC, "-o", BIN + ".tmp",
           "-L", os.path.join(ROOT, "paper_1507_04941_amd"), "-lgsf",
           "-L", os.path.join(ROOT, "oracle"), "-loracle_gsf",
           "-L", "/opt/rocm/lib", "-lamdhip64", "-lm",
           "-Wl,-rpath,$ORIGIN/../../paper_1507_04941_amd:$ORIGIN/../../oracle:/opt/rocm/lib"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    print(build(verbose=True))
