"""The serving loop on the GPU: Poisson arrivals of uneven noise-plus-source
sub-cubes on several streams under an HBM budget.  Each request's results
equal those of the request run alone; the smallest, median and largest
served requests and a few random ones match the FP64 oracle element by
element (FP32 and FP16 storage); requests that can never fit the budget are
rejected with GSF_ERR_BUDGET; the requests in flight never exceed it."""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_04941_amd import binding as B
from paper_1507_04941_amd import serve
from tests.parity import (REL16, REL16_F, check_filtered, check_mask, check_stats, cube_scale,
                          log, sigma_f)

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
FILTERS = [(1.0, 2.0), (2.0, 8.0), (4.0, 2.0)]
BOX = (16, 16, 32)
K = 4.0


def _requests(n, arr, dtype=torch.float32):
    t, shapes = arr.draw(n)
    return [serve.Request(j, float(t[j]), serve.device_cube(shapes[j], arr.cube_seed + j, DEV,
                                                            dtype))
            for j in range(n)]


def _serve(reqs, budget=200e9, lanes=4):
    big = max(reqs, key=lambda r: r.voxels).cube.shape
    srv = serve.Server(FILTERS, BOX, K, lanes=lanes, budget_bytes=budget, max_shape=big,
                       device=DEV, dtype=reqs[0].cube.dtype)
    kept = {}

    def collect(r):
        with torch.cuda.stream(srv.streams[r.lane]):
            kept[r.rid] = {k: [t.clone() for t in getattr(r, k)]
                           for k in ("masks", "F", "mean", "std")}

    stats = srv.run(reqs, collect=collect)
    torch.cuda.synchronize()
    return srv, stats, kept


def _oracle_check(r, out, name):
    """Every voxel of F, mean, std and mask of a served request against the
    oracle run on the request's own (FP32, or 16-bit-rounded) cube."""
    d = r.cube.float().cpu().numpy()
    ref = oracle.find(d, FILTERS, BOX, K, want_F=True, want_stats=True)
    scale = cube_scale(d)
    rel_f = 1e-5 if name == "f32" else REL16_F[name]
    rel = 1e-5 if name == "f32" else REL16[name]
    worst = []
    for j, f in enumerate(FILTERS):
        wf = check_filtered(out["F"][j].float().cpu().numpy(), ref["F"][j], f, scale,
                            what=f"request {r.rid} F[{j}]", rel=rel_f)
        wm, ws = check_stats(out["mean"][j].cpu().numpy(), out["std"][j].cpu().numpy(),
                             ref["mean"][j], ref["std"][j], sigma_f(f) * scale,
                             what=f"request {r.rid} stats[{j}]", rel=rel)
        band = check_mask(B.unpack_mask(out["masks"][j], d.shape), ref["F"][j], ref["mean"][j],
                          ref["std"][j], K, f, scale, what=f"request {r.rid} mask[{j}]",
                          rel=rel, rel_f=rel_f)
        worst.append((wf, wm, ws, band))
    return worst


@pytest.mark.parametrize("name", ["f32", "f16"])
def test_served_results_match_oracle_and_lone_runs(name):
    dt = torch.float32 if name == "f32" else torch.float16
    arr = serve.Arrivals(rate_per_s=3000.0, median_voxels=2.0 ** 17, vmax=2.0 ** 21)
    reqs = _requests(40, arr, dt)
    srv, stats, kept = _serve(reqs)
    log(f"{name}: {stats['requests']} requests p50 {stats['p50_ms']:.2f} ms "
        f"p99 {stats['p99_ms']:.2f} ms, at most {srv.max_busy} in flight")
    assert stats["requests"] == len(reqs) and stats["rejected"] == 0
    assert srv.max_in_flight <= srv.request_budget
    # every request: identical to a lone run of the same cube
    for r in reqs:
        one = B.find(r.cube, FILTERS, BOX, K, want_F=True, want_stats=True)
        for j in range(len(FILTERS)):
            assert torch.equal(kept[r.rid]["masks"][j], one["mask"][0][j]), (r.rid, j)
            assert torch.equal(kept[r.rid]["F"][j], one["F"][0][j]), (r.rid, j)
            assert torch.equal(kept[r.rid]["mean"][j], one["mean"][0][j]), (r.rid, j)
            assert torch.equal(kept[r.rid]["std"][j], one["std"][0][j]), (r.rid, j)
    # smallest, median, largest and three random served requests: the oracle
    by_size = sorted(reqs, key=lambda r: (r.voxels, r.rid))
    rng = np.random.default_rng(11)
    picks = {by_size[0].rid, by_size[len(by_size) // 2].rid, by_size[-1].rid}
    picks |= {int(i) for i in rng.choice(len(reqs), size=3, replace=False)}
    for rid in sorted(picks):
        r = reqs[rid]
        worst = _oracle_check(r, kept[rid], name)
        log(f"  request {rid} {tuple(r.cube.shape)}: " + "; ".join(
            f"F {a:.3g} mean {b:.3g} std {c:.3g} band {n}" for a, b, c, n in worst))
    # the sources are there: some voxel is selected in most requests
    hits = sum(int(any(bool(m.any()) for m in kept[r.rid]["masks"])) for r in reqs)
    assert hits > len(reqs) // 2


def test_tight_budget_serialises_and_rejects():
    arr = serve.Arrivals(rate_per_s=3000.0, median_voxels=2.0 ** 17, vmax=2.0 ** 21, seed=2001)
    reqs = _requests(30, arr)
    nf = len(FILTERS)
    needs = sorted(r.kept_bytes(nf, True) for r in reqs)
    big = max(reqs, key=lambda r: r.voxels).cube.shape
    probe = torch.empty(big, dtype=torch.float32, device=DEV)
    ws = B.find_workspace_size([probe], FILTERS, BOX)
    del probe
    lanes = 3
    # room for the median request alone: larger ones are rejected, the rest
    # run one at a time
    budget = lanes * ws + needs[len(needs) // 2] + 1
    srv, stats, kept = _serve(reqs, budget=budget, lanes=lanes)
    rej = [r for r in reqs if r.status == B.GSF_ERR_BUDGET]
    over = [r for r in reqs if r.kept_bytes(nf, True) > srv.request_budget]
    log(f"budget {budget:.3g}: {stats['requests']} served, {len(rej)} rejected, "
        f"at most {srv.max_busy} in flight")
    assert {r.rid for r in rej} == {r.rid for r in over} and rej
    assert stats["requests"] == len(reqs) - len(rej)
    assert srv.max_in_flight <= srv.request_budget
    for r in rej:
        assert r.rid not in kept
    for r in reqs:
        if r.status == B.GSF_OK:
            one = B.find(r.cube, FILTERS, BOX, K)
            for j in range(nf):
                assert torch.equal(kept[r.rid]["masks"][j], one["mask"][0][j]), (r.rid, j)


def test_latencies_are_after_arrivals():
    arr = serve.Arrivals(rate_per_s=1000.0, median_voxels=2.0 ** 16, vmax=2.0 ** 19)
    reqs = _requests(30, arr)
    big = max(reqs, key=lambda r: r.voxels).cube.shape
    srv = serve.Server(FILTERS, BOX, K, lanes=2, max_shape=big, device=DEV, keep_outputs=False)
    stats = srv.run(reqs)
    for r in reqs:
        assert r.done_s > r.arrival_s and r.start_s >= r.arrival_s
    log(f"p50 {stats['p50_ms']:.2f} ms p99 {stats['p99_ms']:.2f} ms")
