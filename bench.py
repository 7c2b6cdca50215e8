#!/usr/bin/env python3
"""Benchmark of the plain sine-cosine form on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

One step = one pass of the whole hot path (scale/reduce, series, two
doublings, magnitude fix; 4 bytes read and 8 bytes written per element) over
268,435,456 fp32 angles (half uniform in [-pi, pi), half in [-1e4, 1e4),
shuffled, seed 1), resident in HBM before timing starts.  Prints one JSON line.

Roofline: algorithmic bytes per launch = 12 * n; the kernel's average launch
duration comes from HIP events recorded on the stream the kernel runs on,
around the timed launches.  The same traffic with no arithmetic (a 1-read /
2-write float4 copy, same launch shape) gives the measured ceiling.
The CPU baseline is the oracle (plain scalar C) on this host's cores over the
same array.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
BYTES_PER_ELEM = 12
METRIC = "sincos Gelem/s & % HBM roofline (fp32, 1 GPU); p50/p99 latency served"
PMC_FILE = os.path.join(ROOT, "profiles", "plain_sincos_268M_pmc.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_cs_0406049_amd", "csrc", f)
                  for f in ("kernels.hip", "sincos_core.hpp")]


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def counter_traffic(n: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None if there is none or the kernel sources changed since it was taken."""
    try:
        with open(PMC_FILE) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_source_sha256") != kernel_source_hash() or d.get("n") != n:
        return None
    return d.get("hbm_bytes_per_launch")


def time_launches(torch, fn, steps: int, warmup: int):
    """Run fn() warmup times, then time `steps` launches with HIP events on
    torch's current stream (the stream the library launches on) and with the
    host clock.  Returns (event_ms_per_launch, wall_ms_per_launch)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for _ in range(steps):
        fn()
    end.record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) * 1e3 / steps
    return start.elapsed_time(end) / steps, wall


def cpu_baseline(x_host, arith: int):
    """The oracle as it stands over the same array on this host's cores."""
    import oracle
    threads = oracle.default_threads()
    oracle.sincos(x_host[:1 << 16], arith, 0, threads=threads)  # load + warm
    t0 = time.perf_counter()
    oracle.sincos(x_host, arith, 0, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": x_host.size / dt / 1e9, "unit": "Gelem/s", "cores": threads,
            "kind": "oracle",
            "sample": "the full %d-element array, one pass, %s arithmetic, %d threads over "
                      "contiguous chunks (%.2f s wall)" % (x_host.size, ["fused", "split"][arith],
                                                           threads, dt)}


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=1 << 28)
    ap.add_argument("--arith", choices=["fused", "split"], default="fused")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceiling", action="store_true")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the plain form shards into independent ranges; see the design notes). "
              "Run with --gpus 1.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_cs_0406049_amd import _capi, build as hipbuild, workloads

    if not hipbuild.is_built():
        hipbuild.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    _capi.lib()
    props = torch.cuda.get_device_properties(0)
    log("device %s, %d CUs, %s" % (props.name, props.multi_processor_count, _capi.version()))

    n = args.n
    log("generating %d angles" % n)
    if n == 1 << 28:
        x_host = workloads.plain_roofline(n)
        wl = ("plain sincos: 268,435,456 fp32 angles, half U[-pi,pi), half U[-1e4,1e4), "
              "shuffled, seed 1 (1 GiB in, 2 GiB out)")
    else:
        x_host = workloads.uniform_angles(n, -1e4, 1e4, seed=1)
        wl = "plain sincos: %d fp32 angles U[-1e4,1e4), seed 1" % n
    x = torch.from_numpy(x_host).cuda()
    s = torch.empty_like(x)
    c = torch.empty_like(x)
    arith = 0 if args.arith == "fused" else 1
    launch = None
    if args.block or args.unroll or args.grid:
        launch = (args.block, args.unroll, args.grid)
    torch.cuda.synchronize()

    def step():
        _capi.sincos_f32_ex(x, s, c, n, arith, 0, launch)

    log("timing %d steps after %d warmup" % (args.steps, args.warmup))
    ev_ms, wall_ms = time_launches(torch, step, args.steps, args.warmup)
    value = n / (wall_ms * 1e-3) / 1e9
    achieved = BYTES_PER_ELEM * n / (ev_ms * 1e-3) / 1e9
    log("sincos: %.4f ms/launch (events), %.4f ms/step (wall): %.1f Gelem/s, %.0f GB/s" % (
        ev_ms, wall_ms, value, achieved))

    ceiling = None
    if not args.no_ceiling:
        def copy_step():
            _capi.sincos_copy_ceiling_f32(x, s, c, n, launch)
        cev, _ = time_launches(torch, copy_step, args.steps, args.warmup)
        ceiling = BYTES_PER_ELEM * n / (cev * 1e-3) / 1e9
        log("copy ceiling (1 read : 2 writes): %.4f ms, %.0f GB/s" % (cev, ceiling))
        step()  # leave the sine-cosine outputs in s, c
        torch.cuda.synchronize()

    traffic = counter_traffic(n)
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Gelem/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall_ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wl, "n": n, "bytes_per_elem": BYTES_PER_ELEM,
                   "arith": args.arith, "method": "normalized (first method)",
                   "launch": {"block": args.block or 256, "unroll": args.unroll or 4,
                              "grid": args.grid or "cover"},
                   "device": props.name, "cus": props.multi_processor_count},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic,
                     "kernel": "k_sincos_vec (plain form)",
                     "kernel_ms": round(ev_ms, 5),
                     "measured_ceiling_GBps": None if ceiling is None else round(ceiling, 1)},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(x_host, arith)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
