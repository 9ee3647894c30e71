"""GPU parity at the measured size: the 512x512x1024 cube with the six-filter
bank and 64^3 boxes, in the launch configuration the benchmark times (one
gsf_find over all filters).  Every voxel of F, the local mean and std and the
mask of each filter is compared with the FP64 oracle run on the same cube."""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import synth
from tests.parity import check_filtered, check_mask, check_stats, cube_scale, log, sigma_f

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
W = synth.LARGE


@pytest.fixture(scope="module")
def large():
    log(f"full size: generating {W.name}")
    d = synth.workload_cube(W)
    g = torch.from_numpy(d).to(DEV)
    log("full size: gsf_find masks only (the measured configuration)")
    masks_only = B.find(g, W.filters, W.box, W.k)
    log("full size: gsf_find with F, mean and std")
    full = B.find(g, W.filters, W.box, W.k, want_F=True, want_stats=True)
    torch.cuda.synchronize()
    yield d, masks_only, full
    del masks_only, full, g
    torch.cuda.empty_cache()


def test_masks_only_equals_full_outputs(large):
    _, a, b = large
    for j in range(len(W.filters)):
        assert torch.equal(a["mask"][0][j], b["mask"][0][j]), f"filter {W.filters[j]}"


@pytest.mark.parametrize("j", range(len(W.filters)))
def test_every_voxel_matches_oracle(large, j):
    d, _, out = large
    f = W.filters[j]
    log(f"full size filter {f}: oracle")
    ref = oracle.find(d, [f], W.box, W.k, want_F=True, want_stats=True)
    scale = cube_scale(d)
    log(f"full size filter {f}: compare F")
    wf = check_filtered(out["F"][0][j].cpu().numpy(), ref["F"][0], f, scale)
    log(f"full size filter {f}: compare mean/std")
    wm, ws = check_stats(out["mean"][0][j].cpu().numpy(), out["std"][0][j].cpu().numpy(),
                         ref["mean"][0], ref["std"][0], sigma_f(f) * scale)
    mask_g = B.unpack_mask(out["mask"][0][j], d.shape)
    band = check_mask(mask_g, ref["F"][0], ref["mean"][0], ref["std"][0], W.k, f, scale)
    n_sel = int(mask_g.sum())
    log(f"  F/bound={wf:.3g} mean/bound={wm:.3g} std/bound={ws:.3g} selected={n_sel} "
        f"oracle={int(ref['mask'][0].sum())} band={band}")
    assert n_sel > 0
