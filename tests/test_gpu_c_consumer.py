"""The library from plain C on the GPU: tests/c_abi/find_from_c (built by
__graft_entry__.build()) runs gsf_find over a seeded cube with three filters
through include/gsf.h and the HIP runtime API only, and checks every voxel
of F, mean, std and the masks against the FP64 oracle to the parity bounds,
and that invalid arguments are refused."""
import os
import subprocess

import pytest

from tests.parity import log

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_abi", "find_from_c")


def test_c_caller_matches_oracle():
    if not os.path.exists(BIN):
        raise AssertionError(f"{BIN} is not built; run __graft_entry__.build()")
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=120)
    log(r.stdout.strip())
    assert r.returncode == 0, r.stdout + r.stderr
    assert "c consumer ok" in r.stdout
