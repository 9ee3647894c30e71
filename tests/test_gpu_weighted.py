"""GPU parity of the weighted convolution (Eq. 1, normalised form) against the
FP64 oracle: random positive weights, flagged (zero-weight) channels and
regions, unit weights, and voxels without weighted support (exactly 0)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import synth
from tests.parity import check_filtered, cube_scale, log

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(DEV)


def _weights(shape, seed, flag_channels=False, zero_frac=0.0):
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.2, 2.0, size=shape).astype(np.float32)
    if flag_channels:
        w[:, :, shape[2] // 3: shape[2] // 3 + 60] = 0.0    # a flagged band of channels
    if zero_frac:
        w[rng.random(shape) < zero_frac] = 0.0
    return w


@pytest.mark.parametrize("shape,f,kind", [
    ((40, 36, 140), (1.0, 2.0), "random"), ((33, 17, 300), (2.0, 8.0), "flagged"),
    ((20, 24, 77), (1.5, 2.5), "sparse"), ((64, 64, 128), (2.0, 4.0), "unit"),
    ((9, 11, 50), (6.0, 11.0), "random"),       # generic passes
    ((12, 12, 90), (6.0, 1.0), "flagged")])     # compiled spectral pass, generic spatial passes
def test_weighted_matches_oracle(shape, f, kind):
    log(f"weighted shape={shape} filter={f} weights={kind}")
    d = synth.make_cube(shape, n_sources=3, seed=sum(shape))
    if kind == "unit":
        w = np.ones(shape, dtype=np.float32)
    else:
        w = _weights(shape, 1, flag_channels=kind == "flagged",
                     zero_frac=0.5 if kind == "sparse" else 0.0)
    Fg = B.filter3d_weighted(_gpu(d), _gpu(w), f).cpu().numpy()
    Fo = oracle.filter3d_weighted(d, w, *f)
    worst = check_filtered(Fg, Fo, f, cube_scale(d))
    assert np.all(Fg[Fo == 0.0] == 0.0)
    log(f"  worst/bound={worst:.3g}, {int((Fo == 0).sum())} voxels without weighted support")


def test_unsupported_storage_type():
    d = torch.zeros((4, 4, 8), dtype=torch.float16, device=DEV)
    with pytest.raises(ValueError):
        B.filter3d_weighted(d, d, (1.0, 1.0))
