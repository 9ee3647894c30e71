"""GPU parity at the measured size with 16-bit storage: the 512x512x1024
cube rounded to binary16 or bfloat16, the six-filter bank and 64^3 boxes, in
the launch configuration the benchmark times for its FP16 and BF16 lines
(one gsf_find over all filters, the cube and F stored in the 16-bit type,
the spectral intermediate FP32).  Every voxel of F, the local mean and std
and the mask of each filter is compared with the FP64 oracle run on the same
rounded cube, to the 16-bit bounds of the parity helpers, and, for binary16,
with the oracle run on the original FP32 cube, to the end-to-end bounds."""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import synth
from tests.parity import (REL16, REL16_F, check_e2e16, check_filtered, check_mask,
                          check_mask_e2e16, check_stats, cube_scale, log, round16, sigma_f)

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
W = synth.LARGE


TORCH = {"f16": torch.float16, "bf16": torch.bfloat16}


@pytest.fixture(scope="module", params=["f16", "bf16"])
def large16(request):
    name = request.param
    log(f"full size {name}: generating {W.name}")
    d = synth.workload_cube(W)
    d16 = round16(d, name)
    g = torch.from_numpy(d16).to(DEV).to(TORCH[name])
    log(f"full size {name}: gsf_find with F, mean and std")
    out = B.find(g, W.filters, W.box, W.k, want_F=True, want_stats=True)
    torch.cuda.synchronize()
    if name != "f16":
        del d
        d = None
    yield name, d16, out, d
    del out, g
    torch.cuda.empty_cache()


@pytest.mark.parametrize("j", range(len(W.filters)))
def test_every_voxel_matches_oracle_16(large16, j):
    name, d16, out, d = large16
    f = W.filters[j]
    log(f"full size {name} filter {f}: oracle")
    ref = oracle.find(d16, [f], W.box, W.k, want_F=True, want_stats=True)
    scale = cube_scale(d16)
    Fg = out["F"][0][j].to(torch.float32).cpu().numpy()
    wf = check_filtered(Fg, ref["F"][0], f, scale, what=f"F {name}", rel=REL16_F[name])
    wm, ws = check_stats(out["mean"][0][j].cpu().numpy(), out["std"][0][j].cpu().numpy(),
                         ref["mean"][0], ref["std"][0], sigma_f(f) * scale, what=f"stats {name}",
                         rel=REL16[name])
    mask_g = B.unpack_mask(out["mask"][0][j], d16.shape)
    band = check_mask(mask_g, ref["F"][0], ref["mean"][0], ref["std"][0], W.k, f, scale,
                      what=f"mask {name}", rel=REL16[name], rel_f=REL16_F[name])
    log(f"  F/bound={wf:.3g} mean/bound={wm:.3g} std/bound={ws:.3g} "
        f"selected={int(mask_g.sum())} oracle={int(ref['mask'][0].sum())} band={band}")
    assert int(mask_g.sum()) > 0
    if d is not None:
        del ref
        log(f"full size {name} filter {f}: oracle on the FP32 cube")
        e2e = oracle.find(d, [f], W.box, W.k, want_F=True, want_stats=True)
        ee = check_e2e16(Fg, out["mean"][0][j].cpu().numpy(), out["std"][0][j].cpu().numpy(),
                         e2e, 0, name, f"full size {name} filter {f}")
        diff, eband = check_mask_e2e16(mask_g, e2e, 0, W.k, name, f"full size {name} mask {f}")
        log(f"  end to end (local std units): F={ee['F']:.3g} mean={ee['mean']:.3g} "
            f"std={ee['std']:.3g} mask diffs={diff} (all inside the band of {eband})")
