"""GPU parity of the local statistics over the shapes that select the
segmented yz kernel's block forms: z depths on each side of the 3-, 5- and
9-wave choices (2, 4 or 8 output strips of 64 columns per block, with one
halo strip), every power-of-two z window, and y extents that end the y walk
inside different 16-row chunks of its ring turn.  Each case is compared
with the FP64 oracle on the same seeded cube, FP32 and binary16 storage."""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import synth
from tests.parity import REL16, check_stats, cube_scale, log, round16, sigma_f

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FILT = (1.0, 2.0)

# (shape, box): nz 64 / 128 -> 3 waves, 129 / 256 -> 5, 300 / 512 -> 9,
# 600 -> 5 (three blocks of 4 strips walk fewer columns than two of 8),
# 1030 -> 5; ny + by/2 - 1 lands in each quarter of a 64-row turn.
CASES = [
    ((3, 5, 64), (8, 64, 64)),
    ((2, 49, 128), (8, 64, 16)),
    ((3, 17, 129), (16, 16, 32)),
    ((2, 70, 256), (8, 64, 64)),
    ((2, 33, 300), (8, 32, 16)),
    ((2, 97, 512), (8, 64, 32)),
    ((2, 20, 600), (8, 8, 64)),
    ((1, 40, 1030), (8, 64, 64)),
]


def _cube(shape, seed):
    d = synth.make_cube(shape, n_sources=2, seed=seed)
    return (oracle.filter3d(d, *FILT)).astype(np.float32), cube_scale(d)


@pytest.mark.parametrize("shape,box", CASES)
def test_stats_block_forms_fp32(shape, box):
    log(f"stats block forms shape={shape} box={box}")
    Fin, scale = _cube(shape, sum(shape))
    mg, sg = B.local_stats(torch.from_numpy(Fin).to(DEV), box)
    mo, so = oracle.local_stats(Fin.astype(np.float64), box)
    wm, ws = check_stats(mg.cpu().numpy(), sg.cpu().numpy(), mo, so, sigma_f(FILT) * scale)
    log(f"  worst mean/bound={wm:.3g} std/bound={ws:.3g}")


@pytest.mark.parametrize("shape,box", CASES[1::3])
def test_stats_block_forms_fp16(shape, box):
    log(f"stats block forms fp16 shape={shape} box={box}")
    Fin, scale = _cube(shape, sum(shape) + 1)
    F16 = round16(Fin, "f16")
    mg, sg = B.local_stats(torch.from_numpy(Fin).to(DEV).to(torch.float16), box)
    mo, so = oracle.local_stats(F16.astype(np.float64), box)
    wm, ws = check_stats(mg.cpu().numpy(), sg.cpu().numpy(), mo, so, sigma_f(FILT) * scale,
                         what="stats f16", rel=REL16["f16"])
    log(f"  worst mean/bound={wm:.3g} std/bound={ws:.3g}")
