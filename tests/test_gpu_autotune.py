"""The autotuner on the GPU: it tunes a small batch of halo sub-cubes per
size class, caches the winners in JSON, installs them into the library's
table, and the tuned batch still matches the oracle's sub-cube composition
(and gives the same F as the default configuration, bit for bit)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_04941_amd import autotune
from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import synth
from tests.parity import check_filtered, check_mask, check_stats, cube_scale, log, sigma_f

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FILTERS = [(1.0, 2.0), (2.0, 2.0), (4.0, 2.0), (1.0, 4.0)]
BOX = (16, 16, 32)
CASES = [((60, 52, 200), (4, 4, 8)), ((36, 40, 120), (4, 4, 8)), ((70, 30, 90), (2, 2, 4)),
         ((28, 28, 300), (3, 3, 6))]


def test_tune_install_and_parity(tmp_path):
    B.tuning_reset()
    host = [synth.make_cube(s, n_sources=3, seed=900 + i) for i, (s, _) in enumerate(CASES)]
    cubes = [torch.from_numpy(h).to(DEV) for h in host]
    halos = [h for _, h in CASES]
    default = B.find(cubes, FILTERS, BOX, 4.0, want_F=True, halos=halos)
    cache = autotune.tune(cubes, FILTERS, BOX, 4.0, halos=halos, steps=1, reps=1, log=log)
    classes = {B.size_class(B.core_shape(c.shape, h)) for c, h in zip(cubes, halos)}
    dev = autotune.device_name(DEV)
    for cls in classes:
        e = cache[autotune.entry_key(dev, cls, FILTERS, BOX, torch.float32)]
        assert set(e["config"]) == set(autotune.DEFAULT)
        assert len(e["trials"]) >= 4 and e["ms"] > 0
    path = autotune.save(cache, str(tmp_path / "tune.json"))
    again = autotune.load(path)
    assert again == cache
    B.tuning_reset()
    assert autotune.install(again, FILTERS, BOX, torch.float32, DEV) == len(classes)
    for cls in classes:
        want = again[autotune.entry_key(dev, cls, FILTERS, BOX, torch.float32)]["config"]
        assert B.tuning_get(cls, torch.float32) == want
    out = B.find(cubes, FILTERS, BOX, 4.0, want_F=True, want_stats=True, halos=halos)
    for i, (c, h) in enumerate(zip(host, halos)):
        ref = oracle.find_halo(c, h, FILTERS, BOX, 4.0)
        scale = cube_scale(c)
        for j, f in enumerate(FILTERS):
            assert torch.equal(out["F"][i][j], default["F"][i][j]), (i, j)
            Fg = out["F"][i][j].cpu().numpy()
            check_filtered(Fg, ref["F"][j], f, scale, what=f"cube {i} F{f}")
            check_stats(out["mean"][i][j].cpu().numpy(), out["std"][i][j].cpu().numpy(),
                        ref["mean"][j], ref["std"][j], sigma_f(f) * scale, what=f"cube {i} {f}")
            check_mask(B.unpack_mask(out["mask"][i][j], Fg.shape), ref["F"][j], ref["mean"][j],
                       ref["std"][j], 4.0, f, scale, what=f"cube {i} mask{f}")
    B.tuning_reset()
