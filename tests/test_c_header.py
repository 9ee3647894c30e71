"""include/gsf.h is a C header: a C99 program that uses the entry points,
types and constants compiles against it with warnings as errors (no GPU;
the program is only compiled, into a temporary directory)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_c_caller_compiles_against_the_header(tmp_path):
    src = os.path.join(ROOT, "tests", "c_abi", "find_from_c.c")
    out = str(tmp_path / "find_from_c.o")
    r = subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-c",
                        "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                        "-I", "/opt/rocm/include", src, "-o", out],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
