"""Launch-configuration autotuner for the library's tunable kernels.

The library keeps a table of launch configurations (gsf_tuning, see
include/gsf.h) keyed by the size class of a cube's core (floor(log2 voxels))
and its storage type.  This module measures candidate configurations on the
GPU for a workload -- one cube or a batch of sub-cubes with a filter bank --
picks the fastest per size class by coordinate descent, caches the winners in
a JSON file and installs them into the library's table.

Coordinate descent over, in order: the spectral-pass schedule (two sigma_z
groups from one read of the cube, or one pass each), the spatial-sweep form
(merged sweeps in each of the compiled block shapes, or one sweep per
filter), the x split of the sweeps (blocks a sweep aims for), the waves
per block of the yz window-sum kernel, and whether the x walk exits its
last ring turn early.  Each candidate is timed as the median of `reps` timed
rounds of `steps` gsf_find calls after a warm-up; candidates that do not beat
the incumbent by more than `min_gain` (relative) are not taken, so noise does
not move the choice.  Results never depend on the configuration beyond
rounding (the tests check every configuration against the oracle).

Cache key: "<device>|<size class>|<radii>|<box>|<dtype>", radii the sorted
(spatial, spectral) radius pairs of the bank; the value is the gsf_tuning
entry and the times that chose it.  The cache lives at $GSF_TUNE_CACHE, else
~/.cache/gsf/tune.json.
"""
from __future__ import annotations

import json
import math
import os
import statistics
from collections import defaultdict

import torch

from . import binding as B

DEFAULT = {"merge_sweeps": 1, "merged_shape": 0, "sweep_blocks": 512, "yz_waves": 0,
           "pair_spectral": 1, "x_exits": 1}
SWEEP_FORMS = [dict(merge_sweeps=1, merged_shape=0), dict(merge_sweeps=1, merged_shape=1),
               dict(merge_sweeps=1, merged_shape=2), dict(merge_sweeps=1, merged_shape=3),
               dict(merge_sweeps=0, merged_shape=0)]
SWEEP_BLOCKS = [256, 512, 1024, 2048]
YZ_WAVES = [0, 3, 5, 9]
_DT_NAME = {torch.float32: "f32", torch.float16: "f16", torch.bfloat16: "bf16"}


def cache_path() -> str:
    return os.environ.get("GSF_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gsf", "tune.json"))


def device_name(device="cuda:0") -> str:
    return torch.cuda.get_device_name(torch.device(device))


def bank_key(filters, truncate: float = 3.0) -> str:
    rad = sorted((int(math.ceil(truncate * float(f[0]))), int(math.ceil(truncate * float(f[1]))))
                 for f in filters)
    return ",".join(f"{a}/{b}" for a, b in rad)


def entry_key(device: str, size_class: int, filters, box, dtype) -> str:
    bx = "x".join(str(int(v)) for v in (box if not isinstance(box, int) else (box,) * 3))
    return f"{device}|{size_class}|{bank_key(filters)}|{bx}|{_DT_NAME[dtype]}"


def load(path: str | None = None) -> dict:
    path = path or cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def save(cache: dict, path: str | None = None) -> str:
    path = path or cache_path()
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)
    return path


def install(cache: dict, filters, box, dtype, device="cuda:0") -> int:
    """Install every cached entry of this device, bank, box and dtype into the
    library's table; returns how many size classes were set."""
    dev = device_name(device)
    n = 0
    for cls in range(41):
        e = cache.get(entry_key(dev, cls, filters, box, dtype))
        if e is not None:
            B.tuning_set(e["config"], cls, dtype)
            n += 1
    return n


def _time_ms(plan, steps: int, reps: int) -> float:
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    plan.run()
    torch.cuda.synchronize()
    times = []
    for _ in range(reps):
        e0.record()
        for _ in range(steps):
            plan.run()
        e1.record()
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1) / steps)
    return statistics.median(times)


def _tune_class(plan, cls: int, dtype, steps: int, reps: int, min_gain: float, log) -> dict:
    """Coordinate descent for one size class from its current entry; the other
    classes keep theirs.  Returns {"config": ..., "ms": ..., "trials": [...]}."""
    best = B.tuning_get(cls, dtype)
    trials = []

    def measure(cfg):
        B.tuning_set(cfg, cls, dtype)
        ms = _time_ms(plan, steps, reps)
        trials.append({"config": dict(cfg), "ms": round(ms, 4)})
        if log:
            log(f"    class {cls} {cfg}: {ms:.3f} ms")
        return ms

    best_ms = measure(best)
    for axis in ("spectral", "form", "sweep_blocks", "yz_waves", "x_exits"):
        if axis == "spectral":
            cands = [dict(best, pair_spectral=v) for v in (1, 0)]
        elif axis == "x_exits":
            cands = [dict(best, x_exits=v) for v in (1, 0)]
        elif axis == "form":
            cands = [dict(best, **c) for c in SWEEP_FORMS]
        elif axis == "sweep_blocks":
            cands = [dict(best, sweep_blocks=v) for v in SWEEP_BLOCKS]
        else:
            cands = [dict(best, yz_waves=v) for v in YZ_WAVES]
        for cfg in cands:
            if cfg == best:
                continue
            ms = measure(cfg)
            if ms < best_ms * (1.0 - min_gain):
                best, best_ms = cfg, ms
    B.tuning_set(best, cls, dtype)
    return {"config": best, "ms": round(best_ms, 4), "trials": trials}


def tune(cubes, filters, box, k: float, halos=None, steps: int = 3, reps: int = 3,
         min_gain: float = 0.01, cache: dict | None = None, log=None) -> dict:
    """Tune the library for a workload and return the updated cache (not yet
    saved).  `cubes`: device tensors of one storage type (a batch is tuned per
    size class of its cores, each class timed as the sub-batch of its cubes
    while the others keep their entries)."""
    if isinstance(cubes, torch.Tensor):
        cubes = [cubes]
    dtype = cubes[0].dtype
    hs = B._halos(halos, len(cubes))
    by_class = defaultdict(list)
    for c, h in zip(cubes, hs):
        by_class[B.size_class(B.core_shape(c.shape, h))].append((c, h))
    cache = dict(cache or {})
    dev = device_name(cubes[0].device)
    for cls in sorted(by_class, reverse=True):
        members = by_class[cls]
        plan = B.FindPlan([c for c, _ in members], filters, box, k, halos=[h for _, h in members])
        if log:
            log(f"  size class {cls}: {len(members)} cube(s)")
        res = _tune_class(plan, cls, dtype, steps, reps, min_gain, log)
        res["cubes"] = len(members)
        cache[entry_key(dev, cls, filters, box, dtype)] = res
        del plan
    return cache
