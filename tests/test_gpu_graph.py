"""gsf_find captured in a HIP graph (through torch.cuda.graph) and replayed:
the batched form forks onto library streams inside the capture.  Every replay
is compared with the eager result, with eager work and synchronisation
between replays."""
import numpy as np
import pytest
import torch

from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import synth
from tests.parity import log

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.mark.parametrize("ncubes", [1, 5])
def test_captured_find_replays_match_eager(ncubes):
    log(f"graph capture of gsf_find over {ncubes} cube(s)")
    shapes = [(40, 36, 140), (27, 50, 80), (70, 20, 200), (16, 16, 52), (30, 33, 300)][:ncubes]
    halos = [(4, 4, 8), (3, 2, 4), (6, 4, 12), (1, 1, 2), (0, 0, 0)][:ncubes]
    cubes = [torch.from_numpy(synth.make_cube(s, n_sources=3, seed=400 + i)).to(DEV)
             for i, s in enumerate(shapes)]
    filters, box = [(1.0, 2.0), (2.0, 4.0)], (8, 8, 16)
    plan = B.FindPlan(cubes, filters, box, 4.0, want_F=True, want_stats=True, halos=halos)
    plan.run()                       # eager, also creates the library streams
    torch.cuda.synchronize()
    eager = {key: [[t.clone() for t in row] for row in getattr(plan, name)]
             for key, name in (("mask", "masks"), ("F", "F"), ("mean", "mean"), ("std", "std"))}
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for grid in (plan.masks, plan.F, plan.mean, plan.std):
            for row in grid:
                for t in row:
                    t.fill_(-1)       # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for key, name in (("mask", "masks"), ("F", "F"), ("mean", "mean"), ("std", "std")):
            for c, row in enumerate(getattr(plan, name)):
                for j, t in enumerate(row):
                    assert torch.equal(t, eager[key][c][j]), (rep, key, c, j)
        log(f"  replay {rep} matches")
