"""The serving loop: Poisson arrivals of uneven sub-cubes on several streams
under an HBM budget.  Each request's results equal those of the request run
alone; admission never lets requests in flight together exceed the budget."""
import numpy as np
import pytest
import torch

from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import serve
from tests.parity import log

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FILTERS = [(1.0, 2.0), (2.0, 8.0), (4.0, 2.0)]
BOX = (16, 16, 32)


def _requests(n, arr):
    t, shapes = arr.draw(n)
    return [serve.Request(j, float(t[j]), serve.device_noise(shapes[j], arr.cube_seed + j, DEV))
            for j in range(n)]


@pytest.mark.parametrize("budget", [200e9, 1e6])
def test_results_same_alone_and_in_the_mix(budget):
    arr = serve.Arrivals(rate_per_s=3000.0, median_voxels=2.0 ** 17, vmax=2.0 ** 21)
    reqs = _requests(40, arr)
    big = max(reqs, key=lambda r: r.voxels).cube.shape
    srv = serve.Server(FILTERS, BOX, 4.0, lanes=4, budget_bytes=budget, max_shape=big, device=DEV)
    kept = {}

    def collect(r):
        with torch.cuda.stream(srv.streams[r.lane]):
            kept[r.rid] = {k: [t.clone() for t in getattr(r, k)]
                           for k in ("masks", "F", "mean", "std")}

    stats = srv.run(reqs, collect=collect)
    torch.cuda.synchronize()
    log(f"budget {budget:.3g}: {stats['requests']} requests p50 {stats['p50_ms']:.2f} ms "
        f"p99 {stats['p99_ms']:.2f} ms, at most {srv.max_busy} in flight, "
        f"{srv.max_in_flight / 1e6:.1f} MB kept together")
    assert stats["requests"] == len(reqs)
    assert srv.max_in_flight <= budget
    if budget < 2e6:
        # every request keeps more than the budget: each runs alone
        assert srv.max_busy == 1
    for r in reqs:
        one = B.find(r.cube, FILTERS, BOX, 4.0, want_F=True, want_stats=True)
        for j in range(len(FILTERS)):
            assert torch.equal(kept[r.rid]["masks"][j], one["mask"][0][j]), (r.rid, j)
            assert torch.equal(kept[r.rid]["F"][j], one["F"][0][j]), (r.rid, j)
            assert torch.equal(kept[r.rid]["mean"][j], one["mean"][0][j]), (r.rid, j)
            assert torch.equal(kept[r.rid]["std"][j], one["std"][0][j]), (r.rid, j)


def test_latencies_are_after_arrivals():
    arr = serve.Arrivals(rate_per_s=1000.0, median_voxels=2.0 ** 16, vmax=2.0 ** 19)
    reqs = _requests(30, arr)
    big = max(reqs, key=lambda r: r.voxels).cube.shape
    srv = serve.Server(FILTERS, BOX, 4.0, lanes=2, max_shape=big, device=DEV, keep_outputs=False)
    stats = srv.run(reqs)
    for r in reqs:
        assert r.done_s > r.arrival_s and r.start_s >= r.arrival_s
    log(f"p50 {stats['p50_ms']:.2f} ms p99 {stats['p99_ms']:.2f} ms")
