"""The serving scheduler on the CPU, driven by a simulated executor and clock
(no GPU): first-come first-served admission, the byte budget never exceeded,
requests that can never fit rejected with GSF_ERR_BUDGET, a failed launch
freeing its lane and bytes without touching the other requests, and the
latency bookkeeping."""
import math

import pytest

from paper_1507_04941_amd import serve


class FakeCube:
    def __init__(self, shape, elem=4):
        self.shape = shape
        self._elem = elem

    def element_size(self):
        return self._elem


class Clock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExecutor:
    """Each request takes `per_voxel` seconds per voxel once launched; the
    launch of any rid in `fail` raises."""

    def __init__(self, clock, per_voxel=1e-9, fail=()):
        self.clock = clock
        self.per_voxel = per_voxel
        self.fail = set(fail)
        self.t0 = None
        self.start = {}
        self.running = set()
        self.peak_lanes = 0
        self.lanes_seen = []

    def begin(self):
        self.t0 = self.clock.now()

    def launch(self, req, lane):
        if req.rid in self.fail:
            raise RuntimeError(f"planted launch failure of request {req.rid}")
        assert lane not in {self.start[r][1] for r in self.running}, "lane double-booked"
        self.start[req.rid] = (self.clock.now() - self.t0, lane)
        self.running.add(req.rid)
        self.peak_lanes = max(self.peak_lanes, len(self.running))
        self.lanes_seen.append(lane)

    def _end(self, req):
        return self.start[req.rid][0] + self.per_voxel * req.voxels

    def finished(self, req):
        fin = self.clock.now() - self.t0 >= self._end(req)
        if fin:
            self.running.discard(req.rid)
        return fin

    def done_time(self, req):
        return self._end(req)


def _requests(n, seed=5, rate=2000.0):
    arr = serve.Arrivals(rate_per_s=rate, median_voxels=2.0 ** 18, vmax=2.0 ** 22, seed=seed)
    t, shapes = arr.draw(n)
    return [serve.Request(j, float(t[j]), FakeCube(shapes[j])) for j in range(n)]


def _run(reqs, lanes, budget, fail=(), keep=True, per_voxel=1e-9):
    clock = Clock()
    ex = FakeExecutor(clock, per_voxel=per_voxel, fail=fail)
    nf = 3
    in_flight = []

    def need(r):
        return r.kept_bytes(nf, keep)

    sch = serve.Scheduler(lanes, budget, ex, need, clock=clock.now, sleep=clock.sleep,
                          poll_s=1e-5)
    orig_launch = ex.launch

    def launch(req, lane):
        orig_launch(req, lane)
        # bytes of every request running at this launch, this one included
        in_flight.append(sum(need(r) for r in reqs if r.rid in ex.running))

    ex.launch = launch
    st = sch.run(reqs)
    return sch, ex, st, in_flight


@pytest.mark.parametrize("budget", [2e8, 5e8, 1e12])
def test_budget_never_exceeded_and_fifo(budget):
    reqs = _requests(200)
    sch, ex, st, in_flight = _run(reqs, lanes=4, budget=budget)
    served = [r for r in reqs if r.status == serve.GSF_OK]
    assert st["requests"] == len(served)
    assert max(in_flight) <= budget
    assert sch.max_in_flight <= budget
    assert ex.peak_lanes <= 4
    # first come, first served: admission follows arrival order
    arrival_order = [r.rid for r in sorted(served, key=lambda r: (r.arrival_s, r.rid))]
    assert sch.admitted == arrival_order
    for r in served:
        assert r.start_s >= r.arrival_s
        assert r.done_s > r.start_s
    if budget >= 1e12:
        assert ex.peak_lanes == 4          # saturated lanes under a loose budget


def test_request_over_budget_is_rejected():
    reqs = _requests(60)
    nf = 3
    needs = sorted(r.kept_bytes(nf, True) for r in reqs)
    budget = needs[-5] + 1                 # the largest few can never fit
    n_over = sum(1 for n in needs if n > budget)
    assert 1 <= n_over <= 4
    sch, ex, st, in_flight = _run(reqs, lanes=3, budget=budget)
    rej = [r for r in reqs if r.status == serve.GSF_ERR_BUDGET]
    assert len(rej) == n_over
    assert st["rejected"] == n_over
    assert all(r.kept_bytes(nf, True) > budget for r in rej)
    assert all(r.rid not in sch.admitted for r in rej)
    assert all(math.isnan(r.start_s) for r in rej)
    assert st["requests"] == len(reqs) - n_over
    assert max(in_flight) <= budget


def test_failed_launch_frees_its_lane():
    reqs = _requests(40)
    sch, ex, st, _ = _run(reqs, lanes=2, budget=1e12, fail=(3, 17))
    failed = [r for r in reqs if r.status != serve.GSF_OK]
    assert sorted(r.rid for r in failed) == [3, 17]
    assert all("planted" in r.error for r in failed)
    assert st["failed"] == 2
    assert st["requests"] == 38            # everyone else is served
    assert 3 in sch.admitted and 17 in sch.admitted
    assert ex.peak_lanes <= 2


def test_single_lane_serialises():
    reqs = _requests(30)
    sch, ex, st, _ = _run(reqs, lanes=1, budget=1e12)
    assert ex.peak_lanes == 1
    done = sorted(reqs, key=lambda r: r.start_s)
    for a, b in zip(done, done[1:]):
        assert b.start_s >= a.done_s - 1e-9   # one at a time


def test_latency_percentiles():
    reqs = _requests(100)
    _, _, st, _ = _run(reqs, lanes=4, budget=1e12)
    assert 0 < st["p50_ms"] <= st["p99_ms"]
    lat = sorted((r.done_s - r.arrival_s) * 1e3 for r in reqs)
    assert abs(st["mean_ms"] - sum(lat) / len(lat)) < 1e-6
