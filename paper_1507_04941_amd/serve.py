"""Serving loop for the source finder: requests (one sub-cube each) arrive over
time and run through gsf_find on a small set of HIP streams.

Admission is first-come first-served under an HBM budget: a request is
admitted when a stream is free and the bytes it keeps on the device (its
cube, its masks and its device-resident F, local mean and std) fit in the
budget next to the requests in flight; a request that does not fit waits,
and nothing behind it overtakes it.  Streams pick up admitted requests as
they free up (continuous batching: new requests start while others run).
Each stream owns one workspace sized for the largest request.

Latency of a request = its completion on the GPU (a HIP event recorded after
its gsf_find) minus its arrival time, both measured from the start of the
run (a reference event recorded then).  Results of a request do not depend
on what runs beside it.
"""
from __future__ import annotations

import ctypes
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import binding as B


@dataclass
class Request:
    rid: int
    arrival_s: float
    cube: torch.Tensor                       # device-resident input (nx, ny, nz)
    masks: list = field(default_factory=list)
    F: list = field(default_factory=list)
    mean: list = field(default_factory=list)
    std: list = field(default_factory=list)
    start_s: float = math.nan
    done_s: float = math.nan
    lane: int = -1
    end_event: torch.cuda.Event | None = None

    @property
    def voxels(self) -> int:
        return int(self.cube.numel())

    def kept_bytes(self, nfilt: int, keep_outputs: bool) -> int:
        """Device bytes the request holds until it is collected."""
        nx, ny, nz = self.cube.shape
        words = nx * ny * ((nz + 63) // 64)
        b = self.cube.element_size() * self.voxels + 8 * words * nfilt
        if keep_outputs:
            b += (self.cube.element_size() + 8) * self.voxels * nfilt
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


def device_noise(shape, seed: int, device, dtype=torch.float32) -> torch.Tensor:
    """N(0,1) cube made on the device from torch's seeded Philox generator
    (serving inputs; the parity tests use the PCG64 cubes of synth)."""
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return torch.randn(shape, generator=g, device=device, dtype=torch.float32).to(dtype)


class Server:
    """gsf_find over requests on `lanes` streams under an HBM budget."""

    def __init__(self, filters, box, k: float, lanes: int = 4, budget_bytes: float = 200e9,
                 keep_outputs: bool = True, max_shape=None, device="cuda:0",
                 dtype=torch.float32):
        self.filters = [tuple(f) for f in filters]
        self.box = box
        self.k = float(k)
        self.keep = keep_outputs
        self.budget = float(budget_bytes)
        self.device = torch.device(device)
        self.dtype = dtype
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(lanes)]
        self._farr = (B.Filter * len(self.filters))(*[B._filter(f) for f in self.filters])
        self._box = B._box(box)
        # one workspace per lane, sized for the largest request it may serve
        probe = torch.empty(max_shape, dtype=dtype, device=self.device)
        need = B.find_workspace_size([probe], self.filters, box)
        del probe
        self.ws = [torch.empty(need, dtype=torch.uint8, device=self.device) for _ in range(lanes)]
        self.ws_bytes = need

    def _launch(self, req: Request, lane: int) -> None:
        nf = len(self.filters)
        dev = self.device
        shape = tuple(req.cube.shape)
        s = self.streams[lane]
        # outputs belong to the lane's stream: torch's caching allocator hands
        # a freed block only to later work on the same stream, so a released
        # output is never rewritten before the lane's earlier work is done
        with torch.cuda.stream(s):
            req.masks = [B.empty_mask(shape, dev) for _ in range(nf)]
            if self.keep:
                req.F = [torch.empty(shape, dtype=req.cube.dtype, device=dev) for _ in range(nf)]
                req.mean = [torch.empty(shape, dtype=torch.float32, device=dev) for _ in range(nf)]
                req.std = [torch.empty(shape, dtype=torch.float32, device=dev) for _ in range(nf)]
        carr = B._cube_structs([req.cube])

        def ptrs(ts):
            return (B._P * nf)(*[t.data_ptr() for t in ts]) if ts else None

        B._check(B.lib().gsf_find(carr, 1, self._farr, nf, self._box, self.k, ptrs(req.masks),
                                  ptrs(req.F), ptrs(req.mean), ptrs(req.std),
                                  self.ws[lane].data_ptr(), self.ws_bytes, s.cuda_stream))
        req.end_event = torch.cuda.Event(enable_timing=True)
        req.end_event.record(s)
        req.lane = lane

    def run(self, requests: list[Request], collect=None, poll_s: float = 5e-5) -> dict:
        """Serve `requests` (sorted by arrival) in real time; `collect(req)` is
        called when a request completes, after which its outputs are released
        unless the callback keeps them.  Device work the callback issues on
        them belongs on the request's lane stream (``self.streams[req.lane]``),
        which is what orders it before the lane's next request."""
        nf = len(self.filters)
        pending = deque(sorted(requests, key=lambda r: r.arrival_s))
        waiting: deque[Request] = deque()
        busy: dict[int, Request] = {}
        free = list(range(len(self.streams)))
        in_flight = 0.0
        self.max_in_flight = 0.0
        self.max_busy = 0
        done: list[Request] = []
        torch.cuda.synchronize(self.device)
        ref = torch.cuda.Event(enable_timing=True)
        ref.record(torch.cuda.current_stream(self.device))
        t0 = time.perf_counter()
        while pending or waiting or busy:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival_s <= now:
                waiting.append(pending.popleft())
            for lane, req in list(busy.items()):
                if req.end_event.query():
                    req.done_s = ref.elapsed_time(req.end_event) * 1e-3
                    in_flight -= req.kept_bytes(nf, self.keep)
                    del busy[lane]
                    free.append(lane)
                    done.append(req)
                    if collect is not None:
                        collect(req)
                    req.masks, req.F, req.mean, req.std = [], [], [], []
            while waiting and free:
                req = waiting[0]
                need = req.kept_bytes(nf, self.keep)
                if in_flight + need > self.budget and busy:
                    break                              # first come, first served
                waiting.popleft()
                lane = free.pop()
                req.start_s = time.perf_counter() - t0
                self._launch(req, lane)
                in_flight += need
                busy[lane] = req
                self.max_busy = max(self.max_busy, len(busy))
                if len(busy) > 1:
                    self.max_in_flight = max(self.max_in_flight, in_flight)
            if not (pending and pending[0].arrival_s <= time.perf_counter() - t0):
                time.sleep(poll_s)
        wall = time.perf_counter() - t0
        lat = np.array([r.done_s - r.arrival_s for r in done]) * 1e3
        vox = sum(r.voxels for r in done)
        return {
            "requests": len(done),
            "wall_s": wall,
            "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean()),
            "value": vox * nf / max(max(r.done_s for r in done), 1e-9) / 1e9,
            "unit": "GVoxel-filters/s",
        }
