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

Prints one JSON line: GVoxel-filters/s over the timed steps, the dominant
kernel's roofline (algorithmic bytes per launch over its live hipEvent
duration), and the FP64 oracle's rate on the host cores over a bounded
sample of the same workload.
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
                            "gsf_device.h", "gsf_internal.h", "gsf_api.cpp")]


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


def algorithmic_bytes(kernel: str, V: int) -> float | None:
    """Bytes one launch of `kernel` must move for a V-voxel FP32 cube: each
    input read once and each output written once (masks are V/8 bytes)."""
    table = {
        "k_zpass_r": 8.0 * V,          # read d, write T1
        "k_yx_r": 8.0 * V,             # read T1, write F
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


def cpu_baseline(w, d, target_s: float):
    """The FP64 oracle on the host cores over a bounded x-slab of the cube."""
    import numpy as np

    import oracle
    oracle._load()
    threads = oracle.get_threads()
    nx = w.shape[0]

    def run(n):
        sub = np.ascontiguousarray(d[:n])
        t0 = time.perf_counter()
        oracle.find(sub, w.filters, w.box, w.k)
        return time.perf_counter() - t0

    n = min(4, nx)
    t = run(n)
    if t < target_s / 3 and n < nx:
        n = int(min(nx, max(n + 1, n * target_s / max(t, 1e-3))))
        t = run(n)
    vox = n * w.shape[1] * w.shape[2]
    return {
        "value": vox * len(w.filters) / t / 1e9,
        "unit": "GVoxel-filters/s",
        "cores": threads,
        "kind": "oracle",
        "sample": (f"x-slab {n}x{w.shape[1]}x{w.shape[2]} of the same cube, all "
                   f"{len(w.filters)} filters + stats + threshold, FP64, {t:.1f} s wall"),
    }


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


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "small"])
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target wall time of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-storage16", action="store_true",
                    help="skip the FP16/BF16-storage timings")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch of 96 halo sub-cubes")
    ap.add_argument("--serve-requests", type=int, default=400,
                    help="requests of the serving run (Poisson, 200/s); 0 skips it")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration)")
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

    w = synth.LARGE if args.workload == "large" else synth.SMALL
    t0 = time.perf_counter()
    d = synth.workload_cube(w)
    print(f"# generated {w.name} in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    cube = torch.from_numpy(d).to(dev)
    plan = B.FindPlan([cube], w.filters, w.box, w.k)
    V = w.voxels
    for _ in range(args.warmup):
        plan.run()
    torch.cuda.synchronize()
    print(f"# warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    B.profile_reset()
    B.profile_enable(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        plan.run()
    e1.record()
    torch.cuda.synchronize()
    B.profile_enable(False)
    total_ms = e0.elapsed_time(e1)
    kern = B.profile_collect()
    print(f"# timed {args.steps} steps: {total_ms:.2f} ms", file=sys.stderr, flush=True)

    ms_per_step = total_ms / args.steps
    value = V * len(w.filters) / (ms_per_step * 1e-3) / 1e9
    kernels = {k: {"launches": n, "avg_ms": ms / n, "total_ms": ms} for k, (n, ms) in kern.items()}
    dom = max(kern.items(), key=lambda kv: kv[1][1])[0] if kern else None
    roof = None
    if dom is not None:
        n, ms = kern[dom]
        avg_ms = ms / n
        alg = algorithmic_bytes(dom, V)
        sha = kernel_source_sha()
        traffic = read_traffic(dom, w.name, sha)
        if alg is not None:
            ach = alg / (avg_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                    "traffic": traffic, "kernel": dom, "avg_launch_ms": round(avg_ms, 4),
                    "algorithmic_bytes_per_launch": alg, "share_of_step": round(ms / total_ms, 3)}
            if traffic is not None:
                roof["traffic_over_algorithmic"] = round(traffic / alg, 4)
            copy_gbs = copy_bandwidth(dev)
            roof["copy_gbs"] = round(copy_gbs, 1)
            roof["frac_of_copy"] = round(ach / copy_gbs, 4)
            print(f"# device copy: {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
    for k, (n, ms) in kern.items():
        a = algorithmic_bytes(k, V)
        if a is not None:
            kernels[k]["algorithmic_gbs"] = round(a / (ms / n * 1e-3) / 1e9, 1)

    # the same step with the cube, T1 and F stored in 16 bits (window sums FP32)
    storage16 = {}
    if not args.no_storage16:
        for name, dt in (("f16", torch.float16), ("bf16", torch.bfloat16)):
            c16 = cube.to(dt)
            p16 = B.FindPlan([c16], w.filters, w.box, w.k)
            for _ in range(args.warmup):
                p16.run()
            B.profile_reset()
            B.profile_enable(True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(args.steps):
                p16.run()
            e1.record()
            torch.cuda.synchronize()
            B.profile_enable(False)
            t16 = e0.elapsed_time(e1) / args.steps
            k16 = B.profile_collect()
            storage16[name] = {
                "value": round(V * len(w.filters) / (t16 * 1e-3) / 1e9, 3),
                "ms_per_step": round(t16, 4),
                "kernels": {k: {"launches": n, "avg_ms": ms / n} for k, (n, ms) in k16.items()}}
            print(f"# {name} storage: {t16:.3f} ms/step", file=sys.stderr, flush=True)
            del p16, c16

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
        for _ in range(args.warmup):
            B.filter3d_weighted(cube, wts, fw, out=outw, ws=wsw)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            B.filter3d_weighted(cube, wts, fw, out=outw, ws=wsw)
        e1.record()
        torch.cuda.synchronize()
        tw = e0.elapsed_time(e1) / args.steps
        weighted = {"filter": list(fw), "ms_per_call": round(tw, 3),
                    "value": round(V / (tw * 1e-3) / 1e9, 3), "unit": "GVoxel-filters/s"}
        print(f"# weighted: {tw:.3f} ms per call", file=sys.stderr, flush=True)
        del wts, outw, wsw

    # the batched form: 96 uneven sub-cubes with halos in one gsf_find call
    batch = None
    if not args.no_batch:
        bw = synth.BATCH
        t0 = time.perf_counter()
        cubes = [torch.from_numpy(synth.batch_cube(bw, i)).to(dev) for i in range(bw.n_cubes)]
        print(f"# generated {bw.name} in {time.perf_counter() - t0:.1f} s", file=sys.stderr,
              flush=True)
        pb = B.FindPlan(cubes, bw.filters, bw.box, bw.k, halos=bw.halo)
        for _ in range(args.warmup):
            pb.run()
        torch.cuda.synchronize()
        e0.record()
        for _ in range(args.steps):
            pb.run()
        e1.record()
        torch.cuda.synchronize()
        tb = e0.elapsed_time(e1) / args.steps
        core_vox = sum(a * b_ * c for a, b_, c in synth.batch_cores(bw))
        batch = {"workload": bw.name, "cubes": bw.n_cubes, "core_voxels": core_vox,
                 "value": round(core_vox * len(bw.filters) / (tb * 1e-3) / 1e9, 3),
                 "unit": "GVoxel-filters/s", "ms_per_call": round(tb, 3)}
        print(f"# batch: {tb:.2f} ms per call", file=sys.stderr, flush=True)
        del pb, cubes

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
                                  serve.device_noise(shapes[j], arr.cube_seed + j, dev, dt))
                    for j in range(args.serve_requests)]
            big = max(reqs, key=lambda r: r.voxels).cube.shape
            srv = serve.Server(w.filters, w.box, w.k, lanes=4, max_shape=big, device=dev, dtype=dt)
            srv.run(reqs)                                   # warm the allocator
            st = srv.run(reqs)
            serving[name] = {k: round(v, 3) for k, v in st.items() if isinstance(v, float)}
            print(f"# serving {name}: p50 {st['p50_ms']:.2f} ms p99 {st['p99_ms']:.2f} ms",
                  file=sys.stderr, flush=True)
            del reqs, srv
            torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, d, args.cpu_seconds)

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
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
