"""Serving loop for the source finder: requests (one sub-cube each) arrive over
time and run through gsf_find on a small set of HIP streams ("lanes").

Admission is first-come first-served under an HBM budget.  The budget covers
the lanes' workspaces (allocated once, each sized for the largest request)
and, per request in flight or not yet collected, the bytes it keeps on the
device: its cube, its masks and its device-resident F, local mean and std.
A request is admitted when a lane is free and its bytes fit next to those of
the requests in flight; one that does not fit waits, and nothing behind it
overtakes it.  A request that could never fit (its bytes exceed the budget
left after the workspaces) is rejected with GSF_ERR_BUDGET and takes no
lane.  Lanes pick up admitted requests as they free up (continuous batching:
new requests start while others run); a request whose launch fails is marked
with its status and frees its lane and bytes at once.

The scheduling logic (Scheduler) is plain Python over an executor interface,
so it can be driven by a simulated executor without a GPU; GpuExecutor runs
requests through the library.

Latency of a request = its completion on the GPU (a HIP event recorded after
its gsf_find) minus its arrival time, both measured from the start of the
run (a reference event recorded then).  Results of a request do not depend
on what runs beside it.
"""
from __future__ import annotations

import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

GSF_OK = 0
GSF_ERR_BUDGET = 5


@dataclass
class Request:
    rid: int
    arrival_s: float
    cube: object                             # device tensor (nx, ny, nz), or a stand-in
    masks: list = field(default_factory=list)
    F: list = field(default_factory=list)
    mean: list = field(default_factory=list)
    std: list = field(default_factory=list)
    start_s: float = math.nan
    done_s: float = math.nan
    lane: int = -1
    status: int = GSF_OK                     # gsf_status of the request
    error: str = ""
    end_event: object = None

    @property
    def voxels(self) -> int:
        return int(math.prod(int(s) for s in self.cube.shape))

    def kept_bytes(self, nfilt: int, keep_outputs: bool) -> int:
        """Device bytes the request holds until it is collected."""
        nx, ny, nz = (int(s) for s in self.cube.shape)
        words = nx * ny * ((nz + 63) // 64)
        elem = self.cube.element_size()
        b = elem * self.voxels + 8 * words * nfilt
        if keep_outputs:
            b += (elem + 8) * self.voxels * nfilt
        return b


@dataclass(frozen=True)
class Arrivals:
    """Poisson arrivals with lognormal request volumes.

    Inter-arrival gaps ~ Exp(rate) and volumes V = clip(lognormal(ln median,
    sigma_ln), vmin, vmax) from PCG64(seed); shape nx = ny = round((V/2)^(1/3)),
    nz = 2 nx.  Request j's cube is seeded with cube_seed + j."""
    rate_per_s: float = 200.0
    median_voxels: float = 2.0 ** 22
    sigma_ln: float = 6.0 * math.log(2.0) / 3.09
    vmin: float = 2.0 ** 15
    vmax: float = 2.0 ** 28
    seed: int = 2000
    cube_seed: int = 3000

    def draw(self, n: int):
        rng = np.random.Generator(np.random.PCG64(self.seed))
        gaps = rng.exponential(1.0 / self.rate_per_s, size=n)
        vol = np.clip(rng.lognormal(math.log(self.median_voxels), self.sigma_ln, size=n),
                      self.vmin, self.vmax)
        t = np.cumsum(gaps)
        shapes = []
        for v in vol:
            nx = max(1, int(round((v / 2.0) ** (1.0 / 3.0))))
            shapes.append((nx, nx, 2 * nx))
        return t, shapes


# Sources per voxel of a served cube: the batch workload's density.
SOURCE_DENSITY = 2.0 ** -17


def device_cube(shape, seed: int, device, dtype=None):
    """A served request's cube, made on the device with the noise-plus-source
    recipe of the synthetic cubes: N(0,1) noise (torch's seeded Philox
    generator, FP64), then round(V / 2^17) 3-D Gaussian sources whose centre,
    amplitude U[2, 6] and widths s_xy U[1, 3], s_z U[2, 8] are drawn in that
    order from PCG64(seed), each added within +-ceil(4 s) of floor(centre),
    clipped at the faces; cast once to FP32 (then to `dtype` if 16-bit).
    Only the noise generator differs from the host recipe, so the parity
    tests copy the cube back rather than regenerate it."""
    import torch
    nx, ny, nz = (int(s) for s in shape)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    cube = torch.randn((nx, ny, nz), generator=g, device=device, dtype=torch.float64)
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    n_src = int(round(nx * ny * nz * SOURCE_DENSITY))
    for _ in range(n_src):
        x0 = rng.uniform(0.0, nx)
        y0 = rng.uniform(0.0, ny)
        z0 = rng.uniform(0.0, nz)
        amp = rng.uniform(2.0, 6.0)
        s_xy = rng.uniform(1.0, 3.0)
        s_z = rng.uniform(2.0, 8.0)
        hxy = int(math.ceil(4.0 * s_xy))
        hz = int(math.ceil(4.0 * s_z))
        cx, cy, cz = int(math.floor(x0)), int(math.floor(y0)), int(math.floor(z0))
        xa, xb = max(cx - hxy, 0), min(cx + hxy + 1, nx)
        ya, yb = max(cy - hxy, 0), min(cy + hxy + 1, ny)
        za, zb = max(cz - hz, 0), min(cz + hz + 1, nz)
        if xa >= xb or ya >= yb or za >= zb:
            continue
        f64 = dict(device=device, dtype=torch.float64)
        ex = torch.exp(-((torch.arange(xa, xb, **f64) - x0) ** 2) / (2.0 * s_xy * s_xy))
        ey = torch.exp(-((torch.arange(ya, yb, **f64) - y0) ** 2) / (2.0 * s_xy * s_xy))
        ez = torch.exp(-((torch.arange(za, zb, **f64) - z0) ** 2) / (2.0 * s_z * s_z))
        cube[xa:xb, ya:yb, za:zb] += amp * ex[:, None, None] * ey[None, :, None] * ez[None, None, :]
    out = cube.to(torch.float32)
    del cube
    if dtype is not None and dtype != torch.float32:
        out = out.to(dtype)
    return out


class Scheduler:
    """First-come first-served admission of requests onto `lanes` lanes under
    a byte budget, with continuous pickup.  The executor runs requests:

      executor.begin()             -- at the start of a run (time reference)
      executor.launch(req, lane)   -- start req on lane; may raise (the
                                      request then fails: status and error
                                      set, lane and bytes freed at once)
      executor.finished(req)       -- True once req's work is complete
      executor.done_time(req)      -- its completion time in s from begin()

    `need(req)` gives the bytes a request keeps until it is collected;
    `budget` is what the requests may keep together."""

    def __init__(self, lanes: int, budget: float, executor, need, clock=time.perf_counter,
                 sleep=time.sleep, poll_s: float = 5e-5):
        if lanes < 1:
            raise ValueError("need at least one lane")
        self.lanes = lanes
        self.budget = float(budget)
        self.ex = executor
        self.need = need
        self.clock = clock
        self.sleep = sleep
        self.poll_s = poll_s
        self.admitted: list[int] = []          # rids in admission order
        self.max_in_flight = 0.0
        self.max_busy = 0

    def run(self, requests, collect=None) -> dict:
        pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        waiting: deque = deque()
        busy: dict = {}
        free = list(range(self.lanes))
        in_flight = 0.0
        done, rejected, failed = [], [], []
        self.admitted = []
        self.max_in_flight = 0.0
        self.max_busy = 0
        self.ex.begin()
        t0 = self.clock()
        while pending or waiting or busy:
            now = self.clock() - t0
            while pending and pending[0].arrival_s <= now:
                waiting.append(pending.popleft())
            for lane, req in list(busy.items()):
                if self.ex.finished(req):
                    req.done_s = self.ex.done_time(req)
                    in_flight -= self.need(req)
                    del busy[lane]
                    free.append(lane)
                    done.append(req)
                    if collect is not None:
                        collect(req)
                    req.masks, req.F, req.mean, req.std = [], [], [], []
            while waiting and free:
                req = waiting[0]
                need = self.need(req)
                if need > self.budget:
                    waiting.popleft()              # can never fit
                    req.status = GSF_ERR_BUDGET
                    req.error = f"request keeps {need} bytes, budget {self.budget:.0f}"
                    rejected.append(req)
                    continue
                if in_flight + need > self.budget:
                    break                          # first come, first served
                waiting.popleft()
                lane = free.pop()
                req.start_s = self.clock() - t0
                self.admitted.append(req.rid)
                try:
                    self.ex.launch(req, lane)
                except Exception as e:             # the request fails alone
                    req.status = getattr(e, "status", -1)
                    req.error = str(e)
                    req.masks, req.F, req.mean, req.std = [], [], [], []
                    free.append(lane)
                    failed.append(req)
                    continue
                req.lane = lane
                in_flight += need
                busy[lane] = req
                self.max_busy = max(self.max_busy, len(busy))
                self.max_in_flight = max(self.max_in_flight, in_flight)
            if not (pending and pending[0].arrival_s <= self.clock() - t0):
                self.sleep(self.poll_s)
        wall = self.clock() - t0
        lat = np.array([r.done_s - r.arrival_s for r in done]) * 1e3
        out = {
            "requests": len(done),
            "rejected": len(rejected),
            "failed": len(failed),
            "wall_s": wall,
            "unit": "GVoxel-filters/s",
        }
        if len(done):
            out.update({
                "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)),
                "mean_ms": float(lat.mean()),
            })
        self.rejected, self.failed, self.done = rejected, failed, done
        return out


class GpuExecutor:
    """Runs each request through gsf_find on its lane's stream, allocating
    its outputs on that stream (torch's caching allocator hands a freed block
    only to later work on the same stream, so a released output is never
    rewritten before the lane's earlier work is done)."""

    def __init__(self, server: "Server"):
        self.srv = server
        self.ref = None

    def begin(self):
        import torch
        torch.cuda.synchronize(self.srv.device)
        self.ref = torch.cuda.Event(enable_timing=True)
        self.ref.record(torch.cuda.current_stream(self.srv.device))

    def launch(self, req: Request, lane: int):
        import torch

        from . import binding as B
        srv = self.srv
        nf = len(srv.filters)
        dev = srv.device
        shape = tuple(req.cube.shape)
        s = srv.streams[lane]
        with torch.cuda.stream(s):
            req.masks = [B.empty_mask(shape, dev) for _ in range(nf)]
            if srv.keep:
                req.F = [torch.empty(shape, dtype=req.cube.dtype, device=dev) for _ in range(nf)]
                req.mean = [torch.empty(shape, dtype=torch.float32, device=dev) for _ in range(nf)]
                req.std = [torch.empty(shape, dtype=torch.float32, device=dev) for _ in range(nf)]
        carr = B._cube_structs([req.cube])

        def ptrs(ts):
            return (B._P * nf)(*[t.data_ptr() for t in ts]) if ts else None

        B._check(B.lib().gsf_find(carr, 1, srv._farr, nf, srv._box, srv.k, ptrs(req.masks),
                                  ptrs(req.F), ptrs(req.mean), ptrs(req.std),
                                  srv.ws[lane].data_ptr(), srv.ws_bytes, s.cuda_stream))
        req.end_event = torch.cuda.Event(enable_timing=True)
        req.end_event.record(s)

    def finished(self, req: Request) -> bool:
        return req.end_event.query()

    def done_time(self, req: Request) -> float:
        return self.ref.elapsed_time(req.end_event) * 1e-3


class Server:
    """gsf_find over requests on `lanes` streams under an HBM budget."""

    def __init__(self, filters, box, k: float, lanes: int = 4, budget_bytes: float = 200e9,
                 keep_outputs: bool = True, max_shape=None, device="cuda:0", dtype=None):
        import torch

        from . import binding as B
        self.filters = [tuple(f) for f in filters]
        self.box = box
        self.k = float(k)
        self.keep = keep_outputs
        self.device = torch.device(device)
        self.dtype = torch.float32 if dtype is None else dtype
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(lanes)]
        self._farr = (B.Filter * len(self.filters))(*[B._filter(f) for f in self.filters])
        self._box = B._box(box)
        # one workspace per lane, sized for the largest request it may serve
        probe = torch.empty(max_shape, dtype=self.dtype, device=self.device)
        need = B.find_workspace_size([probe], self.filters, box)
        del probe
        self.ws = [torch.empty(need, dtype=torch.uint8, device=self.device) for _ in range(lanes)]
        self.ws_bytes = need
        self.budget = float(budget_bytes)
        # what the requests may keep together: the budget less the workspaces
        self.request_budget = self.budget - lanes * need
        self.max_in_flight = 0.0
        self.max_busy = 0

    def run(self, requests: list[Request], collect=None, poll_s: float = 5e-5) -> dict:
        """Serve `requests` in real time; `collect(req)` is called when a
        request completes, after which its outputs are released unless the
        callback keeps them.  Device work the callback issues on them belongs
        on the request's lane stream (``self.streams[req.lane]``), which is
        what orders it before the lane's next request."""
        nf = len(self.filters)
        sch = Scheduler(len(self.streams), self.request_budget, GpuExecutor(self),
                        lambda r: r.kept_bytes(nf, self.keep), poll_s=poll_s)
        st = sch.run(requests, collect=collect)
        self.max_in_flight = sch.max_in_flight
        self.max_busy = sch.max_busy
        self.admitted = sch.admitted
        self.rejected = sch.rejected
        done = sch.done
        if done:
            vox = sum(r.voxels for r in done)
            st["value"] = vox * nf / max(max(r.done_s for r in done), 1e-9) / 1e9
        return st
