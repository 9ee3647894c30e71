"""gsf_find_noalloc (the entry point for callers that cannot allocate) gives
the same results as gsf_find with a caller workspace: two calls in a row
through the C ABI, the second on a smaller batch, every output compared bit
for bit (both run the same kernels on the same inputs in the same order)."""
import numpy as np
import pytest
import torch

from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import synth
from tests.parity import log

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
# a merged sweep group of three (sigma_z = 2), a pair (sigma_z = 4) and a
# filter alone
FILTERS = [(1.0, 2.0), (2.0, 2.0), (4.0, 2.0), (1.0, 4.0), (2.0, 4.0), (1.0, 1.0)]


def _gpu(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dtype).to(DEV)


def _same(a, b, what):
    for i in range(len(a["mask"])):
        for j in range(len(a["mask"][i])):
            assert torch.equal(a["mask"][i][j], b["mask"][i][j]), f"{what} mask[{i}][{j}]"
            for key in ("F", "mean", "std"):
                if a[key] is not None:
                    assert torch.equal(a[key][i][j], b[key][i][j]), f"{what} {key}[{i}][{j}]"


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_noalloc_matches_find_twice_shrinking(dtype):
    B.init()
    # first call: two cubes with halos, one of them ragged; second: one smaller cube
    first = [synth.make_cube((48, 40, 200), n_sources=5, seed=71),
             synth.make_cube((30, 26, 97), n_sources=2, seed=72)]
    halos = [(4, 4, 8), (2, 3, 5)]
    second = [synth.make_cube((20, 18, 70), n_sources=2, seed=73)]
    box = (16, 8, 32)
    for n, (cubes, hs) in enumerate([(first, halos), (second, [(0, 0, 0)])]):
        log(f"call {n}: {[c.shape for c in cubes]} halos {hs} dtype {dtype}")
        g = [_gpu(c, dtype) for c in cubes]
        ref = B.find(g, FILTERS, box, 4.0, want_F=True, want_stats=True, halos=hs)
        got = B.find_noalloc(g, FILTERS, box, 4.0, want_F=True, want_stats=True, halos=hs)
        torch.cuda.synchronize()
        _same(ref, got, f"call {n}")
        # masks only (the statistics are not written anywhere but the scratch)
        got_m = B.find_noalloc(g, FILTERS, box, 4.0, halos=hs)
        torch.cuda.synchronize()
        for i in range(len(g)):
            for j in range(len(FILTERS)):
                assert torch.equal(ref["mask"][i][j], got_m["mask"][i][j])


def test_noalloc_rejects_a_batch_beyond_the_scratch():
    B.init()
    # 256^3 voxels: one slot needs about 400 MiB with three filters per group
    big = torch.empty((256, 256, 256), dtype=torch.float32, device=DEV)
    with pytest.raises(B.GsfError) as e:
        B.find_noalloc(big, FILTERS[:3], (8, 8, 8), 4.0)
    assert e.value.status == B.GSF_ERR_BUDGET
