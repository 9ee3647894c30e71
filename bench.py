#!/usr/bin/env python3
"""Throughput of the source-finder hot path on one MI355X.

One step = one gsf_find call over the resident 512x512x1024 FP32 cube with the
six-filter bank (sigma_xy in {1,2,4} x sigma_z in {2,8}, truncated at 3 sigma),
64^3 local-statistics boxes and the mean + 4 std selection: every filter is
applied, its local mean/std computed and its mask written.  The cube is in
HBM before the timed region starts; only the masks are produced (the
measured configuration; F, mean and std stay in workspace).  The same step
is then timed with the cube, spectral intermediate and F stored as FP16 and
as BF16 (reported under "storage16"; the headline value is FP32).

Before each timed configuration the library's launch configurations are
autotuned for it (per size class of its cores; reported under "tuning").
The batched form (96 uneven halo sub-cubes, eager and as one captured HIP
graph), the weighted convolution and the serving loop are timed after the
headline.

Prints one JSON line: GVoxel-filters/s over the timed steps, the dominant
kernel's roofline (algorithmic bytes per launch over its live hipEvent
duration), and the FP64 oracle's rate on the host cores over a bounded
sample of the same workload; the same CPU-baseline leg then runs the oracle
on the whole cube, filter by filter, and reports the library's errors
against it for FP32, FP16 and BF16 storage ("errors").
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = ("GVoxel-filters/s + % HBM roofline (FP32 vs FP16-storage); p50/p99 sub-cube latency")
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, vendor figure
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1507_04941_amd", "csrc", n)
                  for n in ("gsf_kernels.hip", "gsf_filter.hip", "gsf_stats.hip",
                            "gsf_merged.h", "gsf_device.h", "gsf_internal.h", "gsf_api.cpp")]


def _code_only(text: str) -> str:
    """Source text without comments and blank lines: what the compiler sees
    (the sources hold no comment markers inside string literals)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    lines = (re.sub(r"//.*", "", line).rstrip() for line in text.splitlines())
    return "\n".join(line for line in lines if line.strip())


def kernel_source_sha() -> str:
    """Hash of the kernel and dispatch sources, comments excluded: a
    counter summary stays valid across comment edits, not across code edits."""
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, encoding="utf-8") as fh:
            h.update(_code_only(fh.read()).encode())
    return h.hexdigest()[:16]


# Algorithmic bytes per voxel-filter, the method's minimum: read the cube
# once and write one mask bit (4 + 1/8 bytes with FP32 storage, 2 + 1/8 with
# 16-bit storage).  A kernel's algorithmic bytes per launch are this figure
# times the voxel-filters the launch serves; the whole step serves
# voxels x filters.
ALG_BYTES_PER_VF = {"f32": 4.125, "f16": 2.125, "bf16": 2.125}


def one_read_bytes_per_vf(storage: str, nfilt: int) -> float:
    """Bytes per voxel-filter if one read of the cube fed every filter and
    each filter wrote its mask bit: (element + nfilt/8) / nfilt."""
    elem = 4.0 if storage == "f32" else 2.0
    return (elem + nfilt / 8.0) / nfilt


def kernel_io_bytes(kernel: str, V: int) -> float | None:
    """Bytes one launch of `kernel` reads and writes for a V-voxel FP32 cube
    in this design (each of its inputs read once, each output written once;
    masks are V/8 bytes).  This counts the design's own intermediates (the
    spectral intermediate, F, the window-sum pairs), unlike ALG_BYTES_PER_VF."""
    table = {
        "k_zpass_r": 8.0 * V,          # read d, write T1
        "k_zpass2_r": 12.0 * V,        # read d, write two T1
        "k_yx_r": 8.0 * V,             # read T1, write F
        "k_yx3_r": 16.0 * V,           # read T1, write three F
        "k_yx2_r": 12.0 * V,           # read T1, write two F
        "k_zpass": 8.0 * V,
        "k_strided_pass": 8.0 * V,     # read T, write T'
        "k_partial_sums": 4.0 * V,     # read F
        "k_box_yz": 12.0 * V,          # read F, write G1, G2
        "k_box_yz_seg": 12.0 * V,
        "k_box_x_select": 12.0 * V + V / 8.0,   # read G1, G2, F, write mask
        "k_zbox": 12.0 * V,            # read F, write Z1, Z2
        "k_ybox": 16.0 * V,            # read Z1, Z2, write Y1, Y2
        "k_xbox_final": 12.0 * V + V / 8.0,   # read Y1, Y2, F, write mask
        "k_threshold": 12.0 * V + V / 8.0,
    }
    kernel = kernel.split("<")[0]
    return table.get(kernel)


def roofline_for(kern: dict, V: int, nfilt: int, steps: int, storage: str,
                 total_ms: float) -> dict | None:
    """The dominant kernel's roofline at the method's algorithmic bytes:
    ALG_BYTES_PER_VF x the voxel-filters one launch serves (voxels x filters
    x steps / its launches) over its mean launch duration."""
    if not kern:
        return None
    dom = max(kern.items(), key=lambda kv: kv[1][1])[0]
    n, ms = kern[dom]
    avg_ms = ms / n
    units = V * nfilt * steps / n
    alg = ALG_BYTES_PER_VF[storage] * units
    ach = alg / (avg_ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(ach / HBM_PEAK_GBS, 4), "kernel": dom,
           "avg_launch_ms": round(avg_ms, 4), "voxel_filters_per_launch": units,
           "algorithmic_bytes_per_launch": alg,
           "share_of_profiled_step": round(ms / total_ms, 3)}
    io = kernel_io_bytes(dom, V) if storage == "f32" else None
    if io is not None:
        io_gbs = io / (avg_ms * 1e-3) / 1e9
        out["kernel_io"] = {"bytes_per_launch": io, "achieved": round(io_gbs, 1),
                            "frac": round(io_gbs / HBM_PEAK_GBS, 4)}
    return out


def traffic_file(kernel: str, workload: str) -> str:
    tag = kernel.replace("<", "_").replace(">", "").replace(",", "_")
    return os.path.join(PROFILES, f"{tag}_{workload}_traffic.txt")


def read_traffic(kernel: str, workload: str, sha: str):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none for this kernel/workload or the kernel sources
    changed since it was taken."""
    path = traffic_file(kernel, workload)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha") != sha:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_model() -> str:
    """The host CPU's model name (first 'model name' of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, d, target_s: float):
    """The FP64 oracle on the host cores over bounded x-slabs of the cube:
    with all the threads it uses by default (about target_s of work), then
    with one thread (about target_s / 2)."""
    import numpy as np

    import oracle
    oracle._load()
    threads = oracle.get_threads()
    nx = w.shape[0]
    plane = w.shape[1] * w.shape[2]

    def run(n):
        sub = np.ascontiguousarray(d[:n])
        t0 = time.perf_counter()
        oracle.find(sub, w.filters, w.box, w.k)
        return time.perf_counter() - t0

    def leg(target):
        n = min(2, nx)
        t = run(n)
        if t < target / 3 and n < nx:
            n = int(min(nx, max(n + 1, n * target / max(t, 1e-3))))
            t = run(n)
        return n, t

    n, t = leg(target_s)
    out = {
        "value": n * plane * len(w.filters) / t / 1e9,
        "unit": "GVoxel-filters/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"x-slab {n}x{w.shape[1]}x{w.shape[2]} of the same cube, all "
                   f"{len(w.filters)} filters + stats + threshold, FP64, {t:.1f} s wall"),
        "cpu_model": cpu_model(),
        "host_cpus": os.cpu_count(),
    }
    try:
        oracle.set_threads(1)
        n1, t1 = leg(target_s / 2)
    finally:
        oracle.set_threads(threads)
    out["one_thread"] = {
        "value": n1 * plane * len(w.filters) / t1 / 1e9,
        "sample": f"x-slab {n1}x{w.shape[1]}x{w.shape[2]}, one thread, {t1:.1f} s wall"}
    return out


def copy_bandwidth(device, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """GB/s (bytes read + written) of a plain 1 GiB device copy: the rate this
    GPU reaches on a streaming kernel, beside the 8 TB/s datasheet peak."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=device).fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * nbytes / (ms * 1e-3) / 1e9


def copy_calibration(device, nbytes: int = 1 << 30, reps: int = 3) -> None:
    """Plain device copy of known size, for scaling rocprofv3 byte counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=device).fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def timed_ms(run, steps: int) -> float:
    """Milliseconds per call of run() over `steps` calls on the current stream,
    bracketed by device synchronisations (library profiling off)."""
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        run()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def profiled(run, steps: int, B) -> tuple[dict, float]:
    """Per-kernel launches and summed milliseconds over `steps` calls, each
    library kernel bracketed by hipEvents on its own stream (a separate pass
    from the headline timing), and the pass's wall time in ms."""
    import torch
    B.profile_reset()
    B.profile_enable(True)
    try:
        ms = timed_ms(run, steps) * steps
    finally:
        B.profile_enable(False)
    kern = B.profile_collect()
    B.profile_reset()
    torch.cuda.synchronize()
    return kern, ms


def kernel_table(kern: dict, V: int) -> dict:
    out = {}
    for k, (n, ms) in kern.items():
        out[k] = {"launches": n, "avg_ms": round(ms / n, 5), "total_ms": round(ms, 4)}
        io = kernel_io_bytes(k, V)
        if io is not None:
            out[k]["io_gbs"] = round(io / (ms / n * 1e-3) / 1e9, 1)
    return out


def noise_sigma_f(f, truncate: float) -> float:
    """sqrt(sum of the squared 3-D taps): the filtered-noise sigma for unit
    input noise (the taps are the sampled unit-sum Gaussians)."""
    import math

    def sumsq(sigma):
        r = int(math.ceil(truncate * sigma))
        g = [math.exp(-(o * o) / (2.0 * sigma * sigma)) for o in range(-r, r + 1)]
        t = sum(g)
        return sum((v / t) ** 2 for v in g)

    return math.sqrt(sumsq(f[0]) ** 2 * sumsq(f[1]))


def unpack_bits(words, shape):
    """Packed mask words (nx, ny, W) on the device -> bool tensor (nx, ny, nz)."""
    import torch
    nx, ny, nz = (int(v) for v in shape)
    b = words.contiguous().view(torch.uint8).reshape(nx, ny, -1, 1)
    bits = (b >> torch.arange(8, device=words.device, dtype=torch.uint8)) & 1
    return bits.reshape(nx, ny, -1)[:, :, :nz].bool()


# End-to-end bounds of each storage type against the FP64 oracle on the FP32
# cube (readings of the parity tests): F within rel_F of max(|F|, unit), mean
# and std within rel_s of unit, unit = the oracle's local std floored at the
# filtered-noise sigma; masks are compared outside the band those bounds span.
E2E_BOUNDS = {"f32": (1e-5, 1e-5), "f16": (1.5e-3, 1e-3), "bf16": (1.6e-2, 8e-3)}


def oracle_errors(B, d, cube32, w, storages) -> dict:
    """Part of the CPU-baseline leg: the FP64 oracle's F, local mean and std of
    every filter on the whole FP32 cube (untimed, after the timed samples),
    against the library's outputs with each storage type, element by element
    on the GPU: per filter the largest errors in units of the local std (and
    of max(|F|, local std) for F), and the mask voxels that differ from the
    oracle's selection, inside and outside the band the storage type's
    bounds span."""
    import torch

    import oracle
    dev = cube32.device
    rms = float(torch.sqrt(torch.mean(cube32.double() ** 2)))
    dts = {"f32": torch.float32, "f16": torch.float16, "bf16": torch.bfloat16}
    per = {name: [] for name in storages}
    t0 = time.perf_counter()
    for f in w.filters:
        ref = oracle.find(d, [f], w.box, w.k, want_F=True, want_stats=True)
        Fo = torch.from_numpy(ref["F"][0]).to(dev)
        mo = torch.from_numpy(ref["mean"][0]).to(dev)
        so = torch.from_numpy(ref["std"][0]).to(dev)
        n_sel_o = int(ref["mask"][0].sum())
        del ref
        unit = torch.clamp(so, min=noise_sigma_f(f, w.truncate) * rms)
        thr = mo + w.k * so
        sel_o = Fo > thr
        scale_f = torch.maximum(Fo.abs(), unit)
        for name in storages:
            rel_f, rel_s = E2E_BOUNDS[name]
            out = B.find(cube32.to(dts[name]), [f], w.box, w.k, want_F=True, want_stats=True)
            torch.cuda.synchronize()
            dF = (out["F"][0][0].double() - Fo).abs()
            e_f = float((dF / unit).max())
            e_fr = float((dF / scale_f).max())
            del dF
            e_m = float(((out["mean"][0][0].double() - mo).abs() / unit).max())
            e_s = float(((out["std"][0][0].double() - so).abs() / unit).max())
            band = (Fo - thr).abs() <= rel_f * scale_f + rel_s * unit + w.k * rel_s * unit
            mg = unpack_bits(out["mask"][0][0], Fo.shape)
            diff = mg != sel_o
            per[name].append({"filter": list(f),
                              "F_max_local_std": round(e_f, 7),
                              "F_max_rel": round(e_fr, 7),
                              "mean_max_local_std": round(e_m, 7),
                              "std_max_local_std": round(e_s, 7),
                              "mask_diffs": int(diff.sum()),
                              "mask_diffs_outside_band": int((diff & ~band).sum()),
                              "band_voxels": int(band.sum()),
                              "selected": int(mg.sum()), "oracle_selected": n_sel_o})
            del out, band, mg, diff
            torch.cuda.empty_cache()
        del Fo, mo, so, unit, thr, sel_o, scale_f
        torch.cuda.empty_cache()
    print(f"# oracle errors in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    return {"against": "the FP64 oracle on the FP32 cube", "unit": "local std",
            "bounds": {k: {"F_rel": v[0], "stats": v[1]} for k, v in E2E_BOUNDS.items()
                       if k in storages},
            "storages": per}


def tune_for(cubes, w, halos=None) -> dict:
    """Autotune the library's launch configurations for one workload (per size
    class of its cores, installed into the library's table for the timed runs
    that follow) and summarise the choice: per class the chosen entry's
    non-default fields and its time against the starting entry's."""
    from paper_1507_04941_amd import autotune
    t0 = time.perf_counter()
    cache = autotune.tune(cubes, w.filters, w.box, w.k, halos=halos, steps=2, reps=3)
    out = {}
    for key, e in sorted(cache.items()):
        cls = key.split("|")[1]
        first = e["trials"][0]
        out[cls] = {"config": {k: v for k, v in e["config"].items()
                               if v != autotune.DEFAULT.get(k)},
                    "ms": e["ms"], "start_ms": first["ms"], "trials": len(e["trials"]),
                    "cubes": e.get("cubes", 1)}
    dt = time.perf_counter() - t0
    print(f"# tuned {len(out)} size class(es) in {dt:.1f} s", file=sys.stderr, flush=True)
    return {"seconds": round(dt, 1), "classes": out}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "small"])
    ap.add_argument("--cpu-seconds", type=float, default=16.0,
                    help="target wall time of the oracle sample with all threads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-storage16", action="store_true",
                    help="skip the FP16/BF16-storage timings")
    ap.add_argument("--no-errors", action="store_true",
                    help="skip the element-wise errors against the FP64 oracle (run with the "
                         "CPU baseline)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch of 96 halo sub-cubes and the weighted form")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="requests of the serving run (Poisson, 200/s); 0 skips it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the library's default launch configurations instead of "
                         "autotuning them first")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by x-slabs with halo exchange; see the design notes)",
              file=sys.stderr, flush=True)
        return 2

    import torch

    from paper_1507_04941_amd import binding as B
    from paper_1507_04941_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a ROCm GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        copy_calibration(dev)
        return 0
    B.init()

    w = synth.LARGE if args.workload == "large" else synth.SMALL
    t0 = time.perf_counter()
    d = synth.workload_cube(w)
    print(f"# generated {w.name} in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    cube = torch.from_numpy(d).to(dev)
    plan = B.FindPlan([cube], w.filters, w.box, w.k)
    V = w.voxels
    nf = len(w.filters)
    tuning = {}
    if not args.no_tune:
        tuning["cube_f32"] = tune_for([cube], w)
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # headline: library profiling off
    ms_per_step = timed_ms(plan.run, args.steps)
    value = V * nf / (ms_per_step * 1e-3) / 1e9
    print(f"# timed {args.steps} steps: {ms_per_step:.3f} ms/step", file=sys.stderr, flush=True)

    # per-kernel durations in a second pass, with hipEvents around each launch
    kern, prof_ms = profiled(plan.run, args.steps, B)
    roof = roofline_for(kern, V, nf, args.steps, "f32", prof_ms)
    if roof is not None:
        sha = kernel_source_sha()
        roof["traffic"] = read_traffic(roof["kernel"], w.name, sha)
        if roof["traffic"] is not None:
            roof["traffic_over_algorithmic"] = round(roof["traffic"] /
                                                     roof["algorithmic_bytes_per_launch"], 3)
        step_gbs = ALG_BYTES_PER_VF["f32"] * V * nf / (ms_per_step * 1e-3) / 1e9
        roof["step"] = {"algorithmic_bytes": ALG_BYTES_PER_VF["f32"] * V * nf,
                        "achieved": round(step_gbs, 1),
                        "frac": round(step_gbs / HBM_PEAK_GBS, 4)}
        one = one_read_bytes_per_vf("f32", nf)
        one_gbs = one * V * nf / (ms_per_step * 1e-3) / 1e9
        roof["step_one_read"] = {"bytes_per_voxel_filter": round(one, 4),
                                 "achieved": round(one_gbs, 1),
                                 "frac": round(one_gbs / HBM_PEAK_GBS, 4)}
        copy_gbs = copy_bandwidth(dev)
        roof["copy_gbs"] = round(copy_gbs, 1)
        print(f"# device copy: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    kernels = kernel_table(kern, V)

    # the same step with the cube and F stored in 16 bits (FP32 spectral
    # intermediate and window sums)
    storage16 = {}
    if not args.no_storage16:
        for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            c16 = cube.to(dt)
            if not args.no_tune:
                tuning[f"cube_{name}"] = tune_for([c16], w)
            p16 = B.FindPlan([c16], w.filters, w.box, w.k)
            for _ in range(args.warmup):
                p16.run()
            t16 = timed_ms(p16.run, args.steps)
            k16, p16_ms = profiled(p16.run, args.steps, B)
            r16 = roofline_for(k16, V, nf, args.steps, name, p16_ms)
            g16 = ALG_BYTES_PER_VF[name] * V * nf / (t16 * 1e-3) / 1e9
            storage16[name] = {
                "value": round(V * nf / (t16 * 1e-3) / 1e9, 3),
                "ms_per_step": round(t16, 4),
                "speedup_vs_f32": round(ms_per_step / t16, 3),
                "roofline": r16,
                "step_frac": round(g16 / HBM_PEAK_GBS, 4),
                "kernels": kernel_table(k16, V)}
            print(f"# {name} storage: {t16:.3f} ms/step", file=sys.stderr, flush=True)
            del p16, c16
            torch.cuda.empty_cache()

    # the weighted convolution (Eq. 1) of the same cube, one filter, random weights
    weighted = None
    if not args.no_batch:
        g = torch.Generator(device=dev)
        g.manual_seed(5)
        wts = torch.rand(cube.shape, generator=g, device=dev) + 0.5
        fw = w.filters[3]
        outw = torch.empty_like(cube)
        n = B._SZ(0)
        B._check(B.lib().gsf_filter3d_weighted_workspace_size(B._dims(cube.shape),
                                                              B.ctypes.byref(B._filter(fw)),
                                                              B.ctypes.byref(n)))
        wsw = torch.empty(int(n.value), dtype=torch.uint8, device=dev)

        def wrun():
            B.filter3d_weighted(cube, wts, fw, out=outw, ws=wsw)

        for _ in range(args.warmup):
            wrun()
        tw = timed_ms(wrun, args.steps)
        weighted = {"filter": list(fw), "ms_per_call": round(tw, 3),
                    "value": round(V / (tw * 1e-3) / 1e9, 3), "unit": "GVoxel-filters/s"}
        print(f"# weighted: {tw:.3f} ms per call", file=sys.stderr, flush=True)
        del wts, outw, wsw
        torch.cuda.empty_cache()

    # the batched form: 96 uneven sub-cubes with halos in one gsf_find call,
    # eager and as one captured HIP graph, FP32 and FP16 storage
    batch = None
    if not args.no_batch:
        bw = synth.BATCH
        t0 = time.perf_counter()
        host = [synth.batch_cube(bw, i) for i in range(bw.n_cubes)]
        print(f"# generated {bw.name} in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
        core_vox = sum(a * b_ * c for a, b_, c in synth.batch_cores(bw))
        batch = {"workload": bw.name, "cubes": bw.n_cubes, "core_voxels": core_vox,
                 "unit": "GVoxel-filters/s"}
        for name, dt in (("f32", torch.float32), ("f16", torch.float16)):
            cubes = [torch.from_numpy(h).to(dev).to(dt) for h in host]
            if not args.no_tune:
                tuning[f"batch_{name}"] = tune_for(cubes, bw, halos=bw.halo)
            pb = B.FindPlan(cubes, bw.filters, bw.box, bw.k, halos=bw.halo)
            for _ in range(args.warmup):
                pb.run()
            tb = timed_ms(pb.run, args.steps)
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph):
                pb.run()
            for _ in range(args.warmup):
                graph.replay()
            tg = timed_ms(graph.replay, args.steps)
            batch[name] = {"value": round(core_vox * nf / (tb * 1e-3) / 1e9, 3),
                           "ms_per_call": round(tb, 3),
                           "graph_value": round(core_vox * nf / (tg * 1e-3) / 1e9, 3),
                           "graph_ms_per_replay": round(tg, 3)}
            print(f"# batch {name}: {tb:.2f} ms per call, {tg:.2f} ms per graph replay",
                  file=sys.stderr, flush=True)
            del graph, pb, cubes
            torch.cuda.empty_cache()
        del host

    # the serving form: Poisson arrivals of lognormal-volume sub-cubes,
    # four streams, 200 GB budget, device-resident F/mean/std
    serving = None
    if args.serve_requests > 0:
        from paper_1507_04941_amd import serve
        arr = serve.Arrivals()
        serving = {"arrivals": f"Poisson {arr.rate_per_s:g}/s, lognormal volume median 2^22, "
                               f"clip [2^15, 2^28], nz = 2 nx = 2 ny",
                   "requests": args.serve_requests}
        for name, dt in (("f32", torch.float32), ("f16", torch.float16)):
            t_arr, shapes = arr.draw(args.serve_requests)
            reqs = [serve.Request(j, float(t_arr[j]),
                                  serve.device_cube(shapes[j], arr.cube_seed + j, dev, dt))
                    for j in range(args.serve_requests)]
            big = max(reqs, key=lambda r: r.voxels).cube.shape
            srv = serve.Server(w.filters, w.box, w.k, lanes=4, max_shape=big, device=dev, dtype=dt)
            srv.run(reqs)                                   # warm the allocator
            st = srv.run(reqs)
            serving[name] = {k: round(v, 3) for k, v in st.items() if isinstance(v, float)}
            serving[name]["rejected"] = st["rejected"]
            print(f"# serving {name}: p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms",
                  file=sys.stderr, flush=True)
            del reqs, srv
            torch.cuda.empty_cache()

    cpu = None
    errors = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, d, args.cpu_seconds)
        if not args.no_errors:
            storages = ["f32"] + ([] if args.no_storage16 else ["f16", "bf16"])
            errors = oracle_errors(B, d, cube, w, storages)

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GVoxel-filters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": f"synthetic: N(0,1) noise + {w.n_sources} Gaussian sources, seed {w.seed}",
        "config": {"workload": w.name, "shape": list(w.shape),
                   "filters": [list(f) for f in w.filters], "truncate": w.truncate,
                   "box": list(w.box), "k": w.k, "storage": "f32", "cubes_per_step": 1,
                   "outputs": "masks"},
        "roofline": roof,
        "cpu_baseline": cpu,
        "kernels": kernels,
        "storage16": storage16 or None,
        "batch": batch,
        "weighted": weighted,
        "serving": serving,
        "tuning": tuning or None,
        "errors": errors,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
