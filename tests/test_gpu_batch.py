"""GPU parity of the batched form: uneven sub-cubes with input-only halos in
one gsf_find call, against the oracle's sub-cube composition (find_halo);
results identical alone and batched; a sub-cube with a halo covering the
filter support reproduces the whole cube's F exactly."""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import synth
from tests.parity import (REL16, REL16_F, check_filtered, check_mask, check_stats, cube_scale,
                          log, round16, sigma_f)

pytestmark = pytest.mark.gpu

DEV = "cuda:0"

# (array shape, halo): thin and wide halos, z halos off the 4-value grid,
# cores below a strip and ragged tails
CASES = [((40, 36, 140), (6, 6, 12)), ((27, 50, 77), (3, 2, 5)), ((70, 20, 200), (12, 4, 24)),
         ((16, 16, 52), (1, 1, 1)), ((30, 33, 300), (0, 0, 0))]
FILTERS = [(1.0, 2.0), (2.0, 2.0), (1.0, 4.0)]


def _gpu(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dtype).to(DEV)


@pytest.mark.parametrize("box", [(8, 16, 32), (5, 7, 9)])
@pytest.mark.parametrize("name", ["f32", "f16"])
def test_halo_subcubes_match_oracle(box, name):
    log(f"batch of {len(CASES)} halo sub-cubes box={box} storage={name}")
    cubes = [synth.make_cube(s, n_sources=3, seed=300 + i) for i, (s, _) in enumerate(CASES)]
    if name != "f32":
        cubes = [round16(c, name) for c in cubes]
    halos = [h for _, h in CASES]
    dt = torch.float32 if name == "f32" else torch.float16
    out = B.find([_gpu(c, dt) for c in cubes], FILTERS, box, 4.0, want_F=True, want_stats=True,
                 halos=halos)
    rel_f = 1e-5 if name == "f32" else REL16_F[name]
    rel = 1e-5 if name == "f32" else REL16[name]
    for i, (c, h) in enumerate(zip(cubes, halos)):
        ref = oracle.find_halo(c, h, FILTERS, box, 4.0)
        scale = cube_scale(c)
        for j, f in enumerate(FILTERS):
            Fg = out["F"][i][j].float().cpu().numpy()
            assert Fg.shape == ref["F"][j].shape
            wf = check_filtered(Fg, ref["F"][j], f, scale, what=f"cube {i} F[{j}]", rel=rel_f)
            wm, ws = check_stats(out["mean"][i][j].cpu().numpy(), out["std"][i][j].cpu().numpy(),
                                 ref["mean"][j], ref["std"][j], sigma_f(f) * scale,
                                 what=f"cube {i} stats[{j}]", rel=rel)
            band = check_mask(B.unpack_mask(out["mask"][i][j], Fg.shape), ref["F"][j],
                              ref["mean"][j], ref["std"][j], 4.0, f, scale,
                              what=f"cube {i} mask[{j}]", rel=rel, rel_f=rel_f)
        log(f"  cube {i} {c.shape} halo {h}: F/bound={wf:.3g} mean/bound={wm:.3g} "
            f"std/bound={ws:.3g} band={band}")


def test_wide_halo_subcube_reproduces_whole_cube():
    log("sub-cube with a halo covering the filter support")
    big = synth.make_cube((64, 60, 256), n_sources=8, seed=21)
    f = (2.0, 4.0)                          # r_xy = 6, r_z = 12
    halo = (6, 8, 12)
    x0, y0, z0, core = 20, 14, 60, (24, 30, 100)
    sub = big[x0 - halo[0]:x0 + core[0] + halo[0], y0 - halo[1]:y0 + core[1] + halo[1],
              z0 - halo[2]:z0 + core[2] + halo[2]]
    Fw = B.filter3d(_gpu(big), f)[x0:x0 + core[0], y0:y0 + core[1], z0:z0 + core[2]]
    Fs = B.find(_gpu(sub), [f], (8, 8, 8), 4.0, want_F=True, halos=halo)["F"][0][0]
    assert torch.equal(Fs, Fw.contiguous())


def test_batch_equals_each_cube_alone():
    b = synth.BATCH
    idx = range(6)
    log(f"first {len(idx)} cubes of {b.name}: batched vs alone")
    cubes = [_gpu(synth.batch_cube(b, i)) for i in idx]
    batch = B.find(cubes, b.filters, b.box, b.k, want_F=True, want_stats=True, halos=b.halo)
    for n, c in enumerate(cubes):
        one = B.find(c, b.filters, b.box, b.k, want_F=True, want_stats=True, halos=b.halo)
        for j in range(len(b.filters)):
            for key in ("mask", "F", "mean", "std"):
                assert torch.equal(batch[key][n][j], one[key][0][j]), (n, j, key)


@pytest.fixture(scope="module")
def batch96():
    b = synth.BATCH
    log(f"generating {b.name}")
    cubes = [_gpu(synth.batch_cube(b, i)) for i in range(b.n_cubes)]
    log("gsf_find over the whole batch (masks only)")
    out = B.find(cubes, b.filters, b.box, b.k, halos=b.halo)
    torch.cuda.synchronize()
    return b, out


@pytest.mark.parametrize("which", ["smallest", "largest", "median"])
def test_batch96_sampled_cubes_match_oracle(batch96, which):
    b, out = batch96
    cores = synth.batch_cores(b)
    order = sorted(range(len(cores)), key=lambda i: np.prod(cores[i]))
    i = {"smallest": order[0], "largest": order[-1], "median": order[len(order) // 2]}[which]
    c = synth.batch_cube(b, i)
    log(f"cube {i} core {cores[i]}: oracle")
    ref = oracle.find_halo(c, b.halo, b.filters, b.box, b.k)
    scale = cube_scale(c)
    for j, f in enumerate(b.filters):
        mask_g = B.unpack_mask(out["mask"][i][j], cores[i])
        band = check_mask(mask_g, ref["F"][j], ref["mean"][j], ref["std"][j], b.k, f, scale,
                          what=f"cube {i} mask[{j}]")
        log(f"  filter {f}: selected {int(mask_g.sum())}, oracle {int(ref['mask'][j].sum())}, "
            f"band {band}")


def test_halo_with_generic_filter_passes():
    # radii beyond the compiled fast paths (r_xy = 18 > 16, r_z = 33 > 32)
    log("halo sub-cube through the generic passes")
    c = synth.make_cube((60, 50, 120), n_sources=3, seed=31)
    halo, f, box = (9, 7, 20), (6.0, 11.0), (8, 8, 16)
    out = B.find(_gpu(c), [f], box, 4.0, want_F=True, want_stats=True, halos=halo)
    ref = oracle.find_halo(c, halo, [f], box, 4.0)
    scale = cube_scale(c)
    wf = check_filtered(out["F"][0][0].cpu().numpy(), ref["F"][0], f, scale)
    wm, ws = check_stats(out["mean"][0][0].cpu().numpy(), out["std"][0][0].cpu().numpy(),
                         ref["mean"][0], ref["std"][0], sigma_f(f) * scale)
    log(f"  F/bound={wf:.3g} mean/bound={wm:.3g} std/bound={ws:.3g}")
