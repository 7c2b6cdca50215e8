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
import math
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
# what determines the plain kernel's code and launch: its arithmetic, the
# streaming helpers, its source and launcher, and the default launch shape
# What the plain kernel's counter figures depend on: its device code and its
# default launch shape (LaunchShape and kBuiltinShape in internal.hpp).
KERNEL_SOURCES = [os.path.join(ROOT, "paper_cs_0406049_amd", "csrc", f)
                  for f in ("sincos_core.hpp", "stream.hpp", "plain.hip")]
LAUNCH_SHAPE_SOURCE = os.path.join(ROOT, "paper_cs_0406049_amd", "csrc", "internal.hpp")
# (block, unroll, grid, lds): lds -1 reserves no LDS, otherwise the bytes each
# workgroup reserves (which caps the workgroups resident per CU)
CEILING_SHAPES = ((64, 1, 0, -1), (64, 1, 0, 7168), (64, 1, 0, 8192), (256, 1, 0, -1))
# memory-traffic probes: (name, probe, shapes tried; the best is reported)
READ_SHAPES = ((1024, 1, 0, -1), (256, 1, 0, -1))
WRITE_SHAPES = ((64, 1, 0, -1), (64, 1, 0, 14336), (64, 1, 0, 16384), (256, 1, 0, -1))
WRITE1_SHAPES = ((256, 1, 0, -1), (64, 1, 0, 16384))


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as f:
            h.update(f.read())
    with open(LAUNCH_SHAPE_SOURCE, "rb") as f:
        text = f.read()
    start = text.index(b"struct LaunchShape {")
    end = text.index(b";", text.index(b"kBuiltinShape[2] =", start)) + 1
    h.update(text[start:end])
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


def time_launches(torch, fn, steps: int, warmup: int, warm_ms: float = 0.0):
    """Run fn() warmup times (and on until warm_ms of wall time has passed),
    then time `steps` launches with HIP events on torch's current stream (the
    stream the library launches on) and with the host clock.  Returns
    (event_ms_per_launch, wall_ms_per_launch).

    warm_ms is for the ALU-bound kernels: after a memory-bound phase the
    shader clock takes some milliseconds of compute to come back up, and a
    short warmup would time part of that ramp instead of the steady state."""
    t_warm = time.perf_counter()
    done = 0
    while done < warmup or (time.perf_counter() - t_warm) * 1e3 < warm_ms:
        fn()
        done += 1
        if done >= warmup and warm_ms > 0 and done % 8 == 0:
            torch.cuda.synchronize()
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
    passes = []
    for _ in range(3):   # three passes over the full array; the median is reported
        t0 = time.perf_counter()
        oracle.sincos(x_host, arith, 0, threads=threads)
        passes.append(time.perf_counter() - t0)
    dt = sorted(passes)[1]
    m = 1 << 25   # single-thread leg: the first 32 Mi elements
    t0 = time.perf_counter()
    oracle.sincos(x_host[:m], arith, 0, threads=1)
    dt1 = time.perf_counter() - t0
    from paper_cs_0406049_amd import workloads
    small = workloads.plain_small()   # the 1,048,576-angle small workload, best of 5
    small_dt = []
    for _ in range(5):
        t0 = time.perf_counter()
        oracle.sincos(small, arith, 0, threads=threads)
        small_dt.append(time.perf_counter() - t0)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return {"value": x_host.size / dt / 1e9, "unit": "Gelem/s", "cores": threads,
            "kind": "oracle", "cpu_model": model, "nproc": os.cpu_count(),
            "small_workload_value": round(small.size / min(small_dt) / 1e9, 5),
            "sample": "the full %d-element array, median of 3 passes, %s arithmetic, %d threads "
                      "over contiguous chunks (%.2f s wall per pass, %.1f thread-seconds in all); "
                      "single thread on its first %d elements: %.4f Gelem/s"
                      % (x_host.size, ["fused", "split"][arith], threads, dt,
                         threads * sum(passes) + dt1, m, m / dt1 / 1e9),
            "single_thread_value": round(m / dt1 / 1e9, 5)}


# ---------------------------------------------------------------------------
# The forms built around the plain kernel, each against its per-call baseline.

# FP32 vector peak 157.3 TFLOP/s counts an FMA as 2 flops: 78.6 T VALU lane-ops
# per second (256 CUs x 128 lanes x 2.4 GHz), each VALU instruction one op.
VALU_PEAK_TOPS = 157.3 / 2
ALU_WARM_MS = 30.0      # compute before timing an ALU-bound kernel (clock ramp)
SERVE_REPLAYS = 5       # open-loop replays of the served workload per configuration
# VALU instructions per (sample, frequency) pair in the one-pass fit step's two
# loops, counted in the gfx950 assembly: 180 per 8 pairs (forward, two samples
# per lane) and 217 per 8 (adjoint, each sample's product r t read with it from
# LDS instead of formed per pair).  The separate forward and adjoint kernels
# take 89 per 4 and 233 per 8.
SINUSOID_FIT_OPS = (180 / 8, 217 / 8)


def bench_ragged(torch, reps, plain_gbs, x_host):
    import numpy as np
    from paper_cs_0406049_amd import _capi, autotune, workloads
    lens, xs_h = workloads.ragged_batch()
    segs = []
    for xh in xs_h:
        x = torch.from_numpy(xh).cuda()
        segs.append((x, torch.empty_like(x), torch.empty_like(x)))
    del xs_h
    elems = int(lens.sum())
    shape, table = autotune.tune_ragged_table(segs, lens, reps=3)

    def best_where(pred):
        for ms, sh in table:
            if pred(sh):
                return {"launch": dict(zip(("block", "unroll", "grid", "lds"), sh)),
                        "kernel_ms": round(ms, 4)}
        return None
    persistent = best_where(lambda sh: sh[2] != autotune.COVER)
    uncapped = best_where(lambda sh: sh[2] == autotune.COVER and sh[3] == -1)
    plan = _capi.RaggedPlan(segs, lens, launch=shape)
    # steady state: a graph launch costs ~15 us more than the bare kernel
    # when launches are back to back, more for the first few
    k_ms, _ = time_launches(torch, plan.launch, max(20, reps), 3)
    # per byte against the plain kernel on the roofline workload, in
    # interleaved A/B rounds (a slow spell of the GPU hits both alike)
    xp = torch.from_numpy(x_host).cuda()
    sp, cp = torch.empty_like(xp), torch.empty_like(xp)
    g_t, p_t = [], []
    for _ in range(5):
        p_t.append(time_launches(torch, lambda: _capi.sincos_f32(xp, sp, cp), max(20, reps), 3)[0])
        g_t.append(time_launches(torch, plan.graph_launch, max(20, reps), 3)[0])
    g_ms, p_ms = float(np.median(g_t)), float(np.median(p_t))
    per_byte_ab = (elems / g_ms) / (xp.numel() / p_ms)
    del xp, sp, cp
    one_ms, _ = time_launches(torch, lambda: _capi.sincos_f32_ragged(segs, lens, launch=shape),
                              reps, 2)
    seg_table = _capi.SegTable(segs, lens)
    tab_ms, _ = time_launches(torch, lambda: _capi.sincos_f32_ragged(seg_table, launch=shape),
                              max(20, reps), 3)

    def per_array():
        for x, s_, c_ in segs:
            _capi.sincos_f32(x, s_, c_, x.numel())
    pa_ms, _ = time_launches(torch, per_array, max(2, reps // 5), 1)
    gbs = BYTES_PER_ELEM * elems / (g_ms * 1e-3) / 1e9
    plan.destroy()
    return {"workload": "4096 arrays, lengths log-uniform in [100, 1e6] (seed 2), %d elements, "
                        "angles U[-100 pi, 100 pi); per byte against the plain kernel on the "
                        "roofline workload in 5 interleaved rounds (medians)" % elems,
            "autotuned_launch": dict(zip(("block", "unroll", "grid", "lds"), shape)),
            "candidates_timed": len(table),
            "best_persistent": persistent, "best_one_per_unit_uncapped": uncapped,
            "graph_ms": round(g_ms, 4), "kernel_ms": round(k_ms, 4),
            "oneshot_staged_ms": round(one_ms, 4),
            "oneshot_segtable_ms": round(tab_ms, 4),
            "oneshot_segtable_vs_graph": round(tab_ms / g_ms, 3),
            "per_array_plain_ms": round(pa_ms, 4),
            "gelem_s": round(elems / (g_ms * 1e-3) / 1e9, 2), "GBps": round(gbs, 1),
            "plain_ms_same_rounds": round(p_ms, 4),
            "per_byte_vs_plain": round(per_byte_ab, 4),
            "per_byte_vs_headline_plain": round(gbs / plain_gbs, 4),
            "speedup_vs_per_array": round(pa_ms / g_ms, 2)}


def memory_ceilings(torch, _capi, x, s, c, n, steps, warmup):
    """What the HBM allows, measured with the library's memory probes (the
    plain kernel's loads and stores with no arithmetic): the 1-read /
    2-write copy in its launch shape (best of a few LDS reservations), the
    same traffic in other schedules, a read-only stream, two and one write
    streams, and the serial bound a perfect alternation of the best read and
    write streams would reach (time = 4n / read rate + 8n / write rate).
    Returns (best 1-read / 2-write GB/s in the plain kernel's schedule,
    references)."""
    P = _capi

    def rate(probe, shape, policy=-1):
        ms, _ = time_launches(torch, lambda: P.sincos_stream_probe_f32(
            probe, x, s, c, n, launch=shape, policy=policy), steps, warmup)
        return P.PROBE_BYTES[probe] * n / (ms * 1e-3) / 1e9

    def best(probe, shapes):
        got = [(rate(probe, sh), sh) for sh in shapes]
        gbs, sh = max(got)
        log("%s: %s" % (P.PROBE_NAMES[probe], ", ".join("%s %.0f" % (b, a) for a, b in got)))
        return round(gbs, 1), dict(zip(("block", "unroll", "grid", "lds"), sh))

    ceiling, ceiling_shape = best(P.PROBE_COPY, CEILING_SHAPES)
    read, read_shape = best(P.PROBE_READ, READ_SHAPES)
    write, write_shape = best(P.PROBE_WRITE, WRITE_SHAPES)
    write1, write1_shape = best(P.PROBE_WRITE1, WRITE1_SHAPES)
    schedules = {}
    for name, probe, shape in (("copy_read_ahead_2", P.PROBE_COPY_BATCH, (64, 2, 0, -1)),
                               ("copy_wave_per_stream", P.PROBE_COPY_SPLIT, (64, 1, 0, -1)),
                               ("copy_wave_per_stream_lds", P.PROBE_COPY_LDS, (64, 1, 0, -1)),
                               ("copy_xcd_contiguous", P.PROBE_COPY_XCD, (64, 1, 0, -1)),
                               ("copy_persistent_8192", P.PROBE_COPY, (64, 1, 8192, -1)),
                               ("copy_nt_sc1_stores", P.PROBE_COPY, (64, 1, 0, -1))):
        schedules[name] = round(rate(probe, shape, 18 if name == "copy_nt_sc1_stores" else -1), 1)
    log("1-read / 2-write schedules: %s" % schedules)
    serial = 12.0 / (4.0 / read + 8.0 / write)
    # references from the runtime and torch: a device-to-device copy
    # (1 read : 1 write) and a fill (writes only), same array size
    cp_ms, _ = time_launches(torch, lambda: s.copy_(x), steps, warmup)
    fill_ms, _ = time_launches(torch, lambda: s.fill_(0.5), steps, warmup)
    refs = {"copy_1r2w_best_shape": ceiling_shape,
            "read_only_GBps": read, "read_only_shape": read_shape,
            "write_only_2streams_GBps": write, "write_only_2streams_shape": write_shape,
            "write_only_1stream_GBps": write1, "write_only_1stream_shape": write1_shape,
            "serial_bound_1r2w_GBps": round(serial, 1),
            "serial_bound_frac_of_peak": round(serial / HBM_PEAK_GBPS, 4),
            "copy_1r2w_frac_of_serial_bound": round(ceiling / serial, 4),
            "other_1r2w_schedules_GBps": schedules,
            "torch_copy_1r1w_GBps": round(8 * n / (cp_ms * 1e-3) / 1e9, 1),
            "torch_fill_write_only_GBps": round(4 * n / (fill_ms * 1e-3) / 1e9, 1)}
    log("references: %s" % refs)
    return ceiling, refs


# the kernels of a counter pass, in dispatch order: (label, call)
COUNTER_PASS = (
    ("plain, no LDS reservation", lambda P, x, s, c, n: P.sincos_f32_ex(x, s, c, n, launch=(64, 1, 0, -1))),
    ("plain, default (7168 B)", lambda P, x, s, c, n: P.sincos_f32_ex(x, s, c, n)),
    ("read probe, 1024 threads", lambda P, x, s, c, n: P.sincos_stream_probe_f32(
        P.PROBE_READ, x, s, None, n, launch=(1024, 1, 0, -1))),
    ("write probe, no reservation", lambda P, x, s, c, n: P.sincos_stream_probe_f32(
        P.PROBE_WRITE, None, s, c, n, launch=(64, 1, 0, -1))),
    ("write probe, 16384 B", lambda P, x, s, c, n: P.sincos_stream_probe_f32(
        P.PROBE_WRITE, None, s, c, n, launch=(64, 1, 0, 16384))),
    ("copy probe, no reservation", lambda P, x, s, c, n: P.sincos_stream_probe_f32(
        P.PROBE_COPY, x, s, c, n, launch=(64, 1, 0, -1))),
    ("copy probe, 8192 B", lambda P, x, s, c, n: P.sincos_stream_probe_f32(
        P.PROBE_COPY, x, s, c, n, launch=(64, 1, 0, 8192))),
)


def counter_pass(torch, _capi, n):
    """Each kernel of COUNTER_PASS three times, in order (uniform angles)."""
    x = torch.rand(n, device="cuda") * 100 - 50
    s = torch.empty_like(x)
    c = torch.empty_like(x)
    for _ in range(3):
        for _label, call in COUNTER_PASS:
            call(_capi, x, s, c, n)
    torch.cuda.synchronize()
    print("counter pass done: %s" % "; ".join(label for label, _ in COUNTER_PASS), flush=True)
    return 0


def bench_variants(torch, reps, x, s, c):
    """The plain kernel with the other arithmetics and the second method, over
    the same roofline arrays (all HBM-bound: the same 12 bytes per element)."""
    import numpy as np
    from paper_cs_0406049_amd import _capi
    n = x.numel()
    res = {"workload": "the roofline workload (%d angles), plain form; A/B rounds against "
                       "the default (fused, first method), median of 3" % n}
    cases = (("fused_method1", 0, 0), ("fused_method2", 0, 1), ("split_method1", 1, 0),
             ("split_method2", 1, 1), ("contract_method1", 2, 0))
    times = {name: [] for name, _, _ in cases}
    for _ in range(3):         # interleaved rounds, so a slow spell hits every case alike
        for name, arith, method in cases:
            ms, _ = time_launches(
                torch, lambda: _capi.sincos_f32_ex(x, s, c, n, arith, method), reps, 3)
            times[name].append(ms)
    base = float(np.median(times["fused_method1"]))
    for name, _, _ in cases[1:]:
        ms = float(np.median(times[name]))
        gbs = BYTES_PER_ELEM * n / (ms * 1e-3) / 1e9
        res[name] = {"kernel_ms": round(ms, 4), "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
                     "GBps": round(gbs, 1), "per_byte_vs_plain": round(base / ms, 4)}
    # one GPU's share if the plain form were split over 8 GPUs: n/8 angles.
    # Successive launches take the 8 shards in turn, so none re-reads data a
    # previous launch left in the 256 MB cache (a shard's traffic is 400 MB).
    m = n // 8
    views = [(x[k * m:(k + 1) * m], s[k * m:(k + 1) * m], c[k * m:(k + 1) * m]) for k in range(8)]
    turn = [0]

    def next_shard():
        xv, sv, cv = views[turn[0] % 8]
        turn[0] += 1
        _capi.sincos_f32(xv, sv, cv, m)
    shard = []
    for _ in range(3):
        shard.append(time_launches(torch, next_shard, 8 * reps, 8)[0])
    ms = float(np.median(shard))
    res["shard_of_8"] = {"n": m, "kernel_ms": round(ms, 4),
                         "gelem_s": round(m / (ms * 1e-3) / 1e9, 2),
                         "per_byte_vs_plain": round(base / (8 * ms), 4)}
    return res


ABLATION_TERMS = {0: (6, 6), 1: (5, 4), 2: (4, 3), 3: (3, 3), 4: (3, 2), 5: (2, 2)}


def bench_ablations(torch, reps, x, s, c):
    """The Sec. II ablations over the roofline arrays, in A/B rounds against
    the plain kernel: the method without its fix, with the text's fix, with
    the eq. (2) doubling, and n = 0..5 doublings after series of the lengths
    the ablation table uses.  All move 12 bytes per element."""
    import numpy as np
    from paper_cs_0406049_amd import _capi
    from paper_cs_0406049_amd.workloads import taylor_series
    n = x.numel()
    cases = [("plain", lambda: _capi.sincos_f32(x, s, c, n), None)]
    for name, v in (("no_fix", _capi.VARIANT_NO_FIX), ("text_fix", _capi.VARIANT_TEXT_FIX),
                    ("eq2_doubling", _capi.VARIANT_EQ2)):
        cases.append((name, lambda v=v: _capi.sincos_f32_variant(x, s, c, n, variant=v), None))
    for nd, (ns, nc) in sorted(ABLATION_TERMS.items()):
        ss, cc = taylor_series(nd, ns, nc)
        cases.append(("doublings_%d_series_%d_%d" % (nd, ns, nc),
                      lambda nd=nd, ss=ss, cc=cc: _capi.sincos_f32_doublings(x, s, c, nd, ss, cc, n),
                      8 + ns + nc + 4 * nd))
    times = {name: [] for name, _, _ in cases}
    for _ in range(3):
        for name, fn, _ in cases:
            ms, _ = time_launches(torch, fn, reps, 3)
            times[name].append(ms)
    base = float(np.median(times["plain"]))
    res = {"workload": "the roofline workload (%d angles); A/B rounds against the plain kernel, "
                       "median of 3" % n}
    for name, _, ops in cases[1:]:
        ms = float(np.median(times[name]))
        res[name] = {"kernel_ms": round(ms, 4), "gelem_s": round(n / (ms * 1e-3) / 1e9, 2),
                     "per_byte_vs_plain": round(base / ms, 4)}
        if ops is not None:
            res[name]["valu_ops_per_element_model"] = ops
    return res


def bench_adjoint(torch, reps, plain_gbs):
    """Elementwise adjoint gx = gs*c - gc*s over the roofline size: 16 bytes
    read and 4 written per element, against the plain kernel's per-byte rate."""
    n = 1 << 28
    g = torch.Generator(device="cuda").manual_seed(5)
    s_ = torch.rand(n, device="cuda", generator=g)
    c_ = torch.rand(n, device="cuda", generator=g)
    gs = torch.rand(n, device="cuda", generator=g)
    gc = torch.rand(n, device="cuda", generator=g)
    gx = torch.empty_like(s_)
    from paper_cs_0406049_amd import _capi
    ms, _ = time_launches(torch, lambda: _capi.sincos_f32_backward(s_, c_, gs, gc, gx, n), reps, 2)
    gbs = 20 * n / (ms * 1e-3) / 1e9
    return {"workload": "gx = gs*c - gc*s, %d elements, both gradients (20 B/element)" % n,
            "kernel_ms": round(ms, 4), "GBps": round(gbs, 1),
            "roofline_frac": round(gbs / HBM_PEAK_GBPS, 4),
            "per_byte_vs_plain": round(gbs / plain_gbs, 4)}


# The pair-ceiling kernel's loop: 208 VALU instructions per trip of 8 pairs.
PAIR_CEILING_OPS = 208 / 8


def valu_ceiling(torch):
    """Measured VALU rate (T lane-ops/s) of the pair's instruction mix with no
    memory traffic: sincos_pair_ceiling_f32 over 2^21 lanes x 256 steps x 8
    chains (several rounds of the chip's resident waves).  Taken right after
    the kernel it is compared with, so both see the same clocks."""
    from paper_cs_0406049_amd import _capi
    n, steps = 1 << 21, 256
    x = torch.rand(n, device="cuda")
    out = torch.empty_like(x)
    ms, _ = time_launches(torch, lambda: _capi.sincos_pair_ceiling_f32(x, out, n, steps), 5, 2,
                          ALU_WARM_MS)
    tops = n * steps * 8 * PAIR_CEILING_OPS / (ms * 1e-3) / 1e12
    log("VALU ceiling (pair mix, no memory): %.3f ms, %.1f T lane-ops/s" % (ms, tops))
    return tops


def alu_roofline(tops, ops_per_pair, ceil):
    return {"bound": "alu", "achieved": round(tops, 2), "peak": round(VALU_PEAK_TOPS, 2),
            "unit": "Tops/s (VALU lane-ops)", "frac": round(tops / VALU_PEAK_TOPS, 4),
            "ops_per_pair": ops_per_pair, "measured_ceiling_Tops": round(ceil, 2),
            "frac_of_measured_ceiling": round(tops / ceil, 4)}


def bench_sinusoid(torch, reps):
    from paper_cs_0406049_amd import _capi, workloads
    from paper_cs_0406049_amd.autograd import (sinusoid_loss_and_grads,
                                               sinusoid_loss_and_grads_two_pass)
    p = workloads.sinusoid_problem()
    d = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    t, A, w, phi, yobs = d(p.t), d(p.A), d(p.w), d(p.phi), d(p.y_obs)
    N, K = t.numel(), A.numel()
    y = torch.empty_like(t)
    f_ms, _ = time_launches(torch, lambda: _capi.sinusoid_f32_forward(t, A, w, phi, y), reps, 2,
                            ALU_WARM_MS)
    r = y - yobs
    gA, gw, gp = torch.empty_like(A), torch.empty_like(A), torch.empty_like(A)
    nb = _capi.sinusoid_f32_backward_workspace_bytes(N, K)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    a_ms, _ = time_launches(torch, lambda: _capi.sinusoid_f32_backward(
        t, r, A, w, phi, gA, gw, gp, ws, nb), reps, 2, ALU_WARM_MS)
    tot_ms, _ = time_launches(torch, lambda: sinusoid_loss_and_grads(t, yobs, A, w, phi), reps, 2,
                              ALU_WARM_MS)
    two_ms, _ = time_launches(torch, lambda: sinusoid_loss_and_grads_two_pass(t, yobs, A, w, phi),
                              reps, 2, ALU_WARM_MS)
    ceil = valu_ceiling(torch)
    # the same fit step captured as a HIP graph (no host work per step)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        sinusoid_loss_and_grads(t, yobs, A, w, phi)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=side):
        sinusoid_loss_and_grads(t, yobs, A, w, phi)
    graph_ms, _ = time_launches(torch, graph.replay, reps, 2, ALU_WARM_MS)
    del graph
    # composed baseline: theta matrix in torch, the plain kernel over it, then
    # rocBLAS products for the model and its gradients
    theta = torch.empty(K, N, device="cuda")
    S = torch.empty_like(theta)
    C = torch.empty_like(theta)

    def composed():
        torch.addcmul(phi[:, None], w[:, None], t[None, :], out=theta)
        _capi.sincos_f32(theta, S, C, theta.numel())
        yy = A @ S
        rr = yy - yobs
        return 0.5 * torch.dot(rr, rr), S @ rr, A * (C @ (rr * t)), A * (C @ rr)
    c_ms, _ = time_launches(torch, composed, reps, 2, ALU_WARM_MS)
    pairs = N * K
    ops = pairs * sum(SINUSOID_FIT_OPS)
    del theta, S, C
    return {"workload": "y(t) = sum_k A_k sin(w_k t + phi_k), N = %d samples, K = %d, loss "
                        "1/2 sum (y - y_obs)^2, forward + adjoint" % (N, K),
            "forward_ms": round(f_ms, 4), "adjoint_ms": round(a_ms, 4),
            "loss_and_grads_ms": round(tot_ms, 4), "loss_and_grads_graph_ms": round(graph_ms, 4),
            "loss_and_grads_two_pass_ms": round(two_ms, 4),
            "composed_plain_kernel_plus_torch_ms":
            round(c_ms, 4), "speedup_vs_composed": round(c_ms / tot_ms, 2),
            "pairs_per_s": round(2 * pairs / (tot_ms * 1e-3), 1),
            "roofline": alu_roofline(ops / (tot_ms * 1e-3) / 1e12, list(SINUSOID_FIT_OPS), ceil)}


def bench_interleaved(torch, reps, plain_gbs, x_host):
    """complex64 (cos, sin) output over the roofline workload: the same 12
    bytes per element in one interleaved stream."""
    from paper_cs_0406049_amd import _capi
    n = x_host.size
    x = torch.from_numpy(x_host).cuda()
    out = torch.empty(2 * n, device="cuda")
    res = {}
    for layout, name in ((0, "complex64"), (1, "phase_blocks")):
        ms, _ = time_launches(torch, lambda: _capi.sincos_f32_interleaved(x, out, n, layout), reps, 2)
        gbs = BYTES_PER_ELEM * n / (ms * 1e-3) / 1e9
        res[name] = {"kernel_ms": round(ms, 4), "GBps": round(gbs, 1),
                     "roofline_frac": round(gbs / HBM_PEAK_GBPS, 4),
                     "per_byte_vs_plain": round(gbs / plain_gbs, 4)}
    res["workload"] = "the roofline workload (%d angles) written as one interleaved array" % n
    return res


HUYGENS_OPS = 90 / 2    # VALU instructions per (point, source) pair in the loop's ISA
# of which v_rsq_f32 and v_rcp_f32 (one each per pair) are transcendental
# instructions, issued at a quarter of the rate of the others: each takes four
# issue slots, so the pair needs 45 + 2 * 3 = 51 slots
HUYGENS_TRANSCENDENTALS = 4 / 2
HUYGENS_SLOTS = HUYGENS_OPS + 3 * HUYGENS_TRANSCENDENTALS


def bench_huygens(torch, reps):
    """Huygens diffraction: 512 x 512 screen points, 64 x 64 sources; the
    fused kernel against the plain kernel composed with torch ops (phase
    matrix in chunks, sincos kernel, weighted sums)."""
    import numpy as np
    from paper_cs_0406049_amd import _capi, workloads
    p = workloads.huygens_problem()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()  # noqa: E731
    xo, yo, src = d(p.xo), d(p.yo), d(p.src.reshape(-1))
    P, S = xo.numel(), p.src.shape[0]
    re = torch.empty_like(xo)
    im = torch.empty_like(xo)
    ms, _ = time_launches(torch, lambda: _capi.huygens_f32(xo, yo, src, p.k, p.L, re, im), reps, 1,
                          ALU_WARM_MS)
    # the term's own ceiling: the same term, lanes and sum length with the
    # sources in registers (8 sources of the table, S / 8 passes)
    src8 = src[:32].clone()
    t_ms, _ = time_launches(torch, lambda: _capi.huygens_term_ceiling_f32(
        xo, yo, src8, S // 8, p.k, p.L, re, im), reps, 1, ALU_WARM_MS)
    ms2, _ = time_launches(torch, lambda: _capi.huygens_f32(xo, yo, src, p.k, p.L, re, im), reps, 1,
                           ALU_WARM_MS)
    ms = min(ms, ms2)
    ceil = valu_ceiling(torch)
    sx, sy, sa, sp = (src.view(S, 4)[:, i] for i in range(4))
    chunk = 1 << 16
    th = torch.empty(chunk, S, device="cuda")
    ss = torch.empty_like(th)
    cc = torch.empty_like(th)
    k32, L32 = float(np.float32(p.k)), float(np.float32(p.L))

    def composed():
        for lo in range(0, P, chunk):
            hi = min(P, lo + chunk)
            dx = xo[lo:hi, None] - sx[None, :]
            dy = yo[lo:hi, None] - sy[None, :]
            rho2 = dx * dx + dy * dy
            r = torch.sqrt(rho2 + L32 * L32)
            torch.mul(rho2 / (r + L32), k32, out=th[:hi - lo])
            th[:hi - lo] += sp[None, :]
            _capi.sincos_f32(th, ss, cc, (hi - lo) * S)
            w = sa[None, :] / r
            re[lo:hi] = (w * cc[:hi - lo]).sum(1)
            im[lo:hi] = (w * ss[:hi - lo]).sum(1)
    c_ms, _ = time_launches(torch, composed, max(2, reps // 4), 1)
    pairs = P * S
    tops = pairs * HUYGENS_OPS / (ms * 1e-3) / 1e12
    return {"workload": "Huygens point-source sum: %d screen points, %d sources (64 x 64 aperture, "
                        "lens + seeded aberration), L = %g wavelengths" % (P, S, p.L),
            "kernel_ms": round(ms, 4), "pairs_per_s": round(pairs / (ms * 1e-3), 1),
            "term_ceiling_ms": round(t_ms, 4),
            "frac_of_term_ceiling": round(t_ms / ms, 4),
            "composed_plain_kernel_plus_torch_ms": round(c_ms, 3),
            "speedup_vs_composed": round(c_ms / ms, 2),
            "roofline": dict(alu_roofline(tops, HUYGENS_OPS, ceil),
                             transcendentals_per_pair=HUYGENS_TRANSCENDENTALS,
                             issue_slots_per_pair=HUYGENS_SLOTS,
                             frac_of_issue_slots=round(
                                 tops * HUYGENS_SLOTS / HUYGENS_OPS / VALU_PEAK_TOPS, 4))}


def bench_serve(torch, plain_gelem_s, only=None):
    import numpy as np
    from paper_cs_0406049_amd import serve, workloads
    rs = workloads.request_stream()
    pool = torch.from_numpy(rs.pool).cuda()
    assert int((rs.offsets + rs.sizes).max()) <= pool.numel()
    xs = [pool.data_ptr() + 4 * int(o) for o in rs.offsets]
    mean_n = float(rs.sizes.mean())
    rate = 0.7 * plain_gelem_s * 1e9 / mean_n
    arr = (np.cumsum(rs.unit_gaps) / rate * 1e9).astype(np.int64)
    arr -= arr[0]
    out = {"workload": "%d requests, sizes log-uniform in [1e3, 1e7] (seed 4, mean %.0f), "
                       "Poisson arrivals at 70%% of the plain kernel's rate (%.0f req/s), "
                       "budget 8 GiB, inputs resident in HBM" % (rs.sizes.size, mean_n, rate)}
    # the batched server with its defaults (size split at 2^22 elements, each
    # class's batches in order on its own stream), the same with every batch
    # on its slot's stream, that without the split, and one plain launch per
    # request.  The batched servers run side by side and take turns: each
    # round replays the 70 % load once on each (order alternating), so drift
    # over the run falls on all alike; SERVE_REPLAYS rounds, and the median
    # and range of each server's p50 and p99 are reported
    variants = (("batched", serve.MODE_BATCHED, 0, False),
                ("batched_stream_per_slot", serve.MODE_BATCHED, 0, True),
                ("batched_no_size_split", serve.MODE_BATCHED, -1, True))
    if only:
        unknown = set(only) - {v[0] for v in variants}
        if unknown:
            raise SystemExit("unknown serve variants: %s" % ", ".join(sorted(unknown)))
        variants = tuple(v for v in variants if v[0] in only)

    def one_run(comp):
        one = serve.latency_summary(comp)
        # where the time goes: waiting to be launched, then on the device
        one["p50_submit_to_launch_us"] = float(
            np.percentile((comp["t_launch_ns"] - comp["t_submit_ns"]) / 1e3, 50))
        one["p50_launch_to_complete_us"] = float(
            np.percentile((comp["t_complete_ns"] - comp["t_launch_ns"]) / 1e3, 50))
        return one

    def saturation(cfg):
        with serve.Server(**cfg) as srv:
            comp = srv.replay(xs, rs.sizes, np.zeros(rs.sizes.size, np.int64))
            return serve.latency_summary(comp)["throughput_gelem_s"]

    cfgs = {name: dict(mode=mode, max_inflight=4, auto_release=True, split_elems=split,
                       stream_per_slot=per_slot) for name, mode, split, per_slot in variants}
    servers = {}
    runs = {name: [] for name in cfgs}
    batches = {}
    try:
        for name, cfg in cfgs.items():
            servers[name] = serve.Server(**cfg)
        for srv in servers.values():
            srv.replay(xs[:200], rs.sizes[:200], np.zeros(200, np.int64))   # warm
        names = list(servers)
        for rnd in range(SERVE_REPLAYS):
            for name in (names if rnd % 2 == 0 else names[::-1]):
                runs[name].append(one_run(servers[name].replay(xs, rs.sizes, arr)))
        for name, srv in servers.items():
            batches[name] = srv.stats()["batches"] // (SERVE_REPLAYS + 1)
    finally:
        for srv in servers.values():
            srv.close()
    cfgs["per_request"] = dict(mode=serve.MODE_PER_REQUEST, max_inflight=4, auto_release=True,
                               stream_per_slot=True)
    with serve.Server(**cfgs["per_request"]) as srv:
        srv.replay(xs[:200], rs.sizes[:200], np.zeros(200, np.int64))   # warm
        runs["per_request"] = [one_run(srv.replay(xs, rs.sizes, arr))]
        batches["per_request"] = srv.stats()["batches"] // 2
    for name, rr in runs.items():
        runs_by_p99 = sorted(rr, key=lambda r: r["p99_us"])
        summ = dict(runs_by_p99[len(rr) // 2])
        summ["batches"] = batches[name]
        if len(rr) > 1:
            for key in ("p50_us", "p99_us"):
                vals = sorted(r[key] for r in rr)
                summ[key + "_median"] = float(np.median(vals))
                summ[key + "_range"] = [round(vals[0], 3), round(vals[-1], 3)]
            summ["replays"] = len(rr)
        sat = saturation(cfgs[name])
        summ["saturation_gelem_s"] = round(sat, 2)
        summ["saturation_per_byte_vs_plain"] = round(sat / plain_gelem_s, 4)
        out[name] = {k: (round(v, 3) if isinstance(v, float) else v) for k, v in summ.items()}
        log("serve %s: p50 %.1f us, p99 %.1f us (median of %d), %.1f Gelem/s delivered, "
            "saturation %.1f" % (name, summ.get("p50_us_median", summ["p50_us"]),
                                 summ.get("p99_us_median", summ["p99_us"]), len(rr),
                                 summ["throughput_gelem_s"], summ["saturation_gelem_s"]))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=40)   # 20 ms: clocks settle
    ap.add_argument("--n", type=int, default=1 << 28)
    ap.add_argument("--arith", choices=["fused", "split"], default="fused")
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--unroll", type=int, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--lds", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ceiling", action="store_true")
    ap.add_argument("--counter-pass", action="store_true",
                    help="only run the plain kernel (with and without its LDS reservation) and "
                         "the read, write and copy probes three times each over the roofline "
                         "workload's size, for rocprofv3 counter runs, then exit")
    ap.add_argument("--forms",
                    default="variants,ablations,ragged,interleaved,adjoint,sinusoid,huygens,serve",
                    help="comma list of forms to measure after the plain kernel ('' = none)")
    ap.add_argument("--serve-variants", default="",
                    help="comma list of the batched servers the serve form measures "
                         "(batched, batched_stream_per_slot, batched_no_size_split; '' = all); "
                         "one plain launch per request is always measured")
    args = ap.parse_args(argv)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the plain form would shard into independent contiguous ranges, one per GPU). "
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
    if args.counter_pass:
        return counter_pass(torch, _capi, n)
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
    if args.block or args.unroll or args.grid or args.lds:
        launch = (args.block, args.unroll, args.grid, args.lds)
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
    references = None
    if not args.no_ceiling:
        ceiling, references = memory_ceilings(torch, _capi, x, s, c, n, args.steps, args.warmup)
        step()  # leave the sine-cosine outputs in s, c
        torch.cuda.synchronize()

    traffic = counter_traffic(n)
    default_plain = _capi.get_tuning()["plain"]
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
                   "launch": {"block": args.block or default_plain["block"],
                              "unroll": args.unroll or default_plain["unroll"],
                              "grid": args.grid or default_plain["grid"] or
                              "one workgroup per tile",
                              "lds_reserved_bytes": max(0, args.lds or default_plain["lds"])},
                   "device": props.name, "cus": props.multi_processor_count},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBPS, 4),
                     "traffic": traffic,
                     "kernel": "k_sincos_vec (plain form)",
                     "kernel_ms": round(ev_ms, 5),
                     "measured_ceiling_GBps": None if ceiling is None else round(ceiling, 1),
                     "frac_of_measured_ceiling": None if ceiling is None else
                     round(achieved / ceiling, 4),
                     "references": references},
    }
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(x_host, arith)
    forms = [f for f in args.forms.split(",") if f]
    if forms:
        out["forms"] = {}
        if "variants" in forms:  # uses the roofline arrays, so before they are freed
            log("form: variants")
            out["forms"]["variants"] = bench_variants(torch, max(10, args.steps // 4), x, s, c)
        if "ablations" in forms:  # also on the roofline arrays
            log("form: ablations")
            out["forms"]["ablations"] = bench_ablations(torch, max(10, args.steps // 4), x, s, c)
        del x, s, c
        torch.cuda.empty_cache()
    for f in forms:
        if f in ("variants", "ablations"):
            continue
        log("form: %s" % f)
        if f == "ragged":
            out["forms"]["ragged"] = bench_ragged(torch, max(5, args.steps // 4), achieved,
                                                  x_host)
        elif f == "interleaved":
            out["forms"]["interleaved"] = bench_interleaved(torch, max(5, args.steps // 4),
                                                            achieved, x_host)
        elif f == "adjoint":
            out["forms"]["adjoint"] = bench_adjoint(torch, max(5, args.steps // 4), achieved)
        elif f == "sinusoid":
            out["forms"]["sinusoid"] = bench_sinusoid(torch, max(20, args.steps))
        elif f == "huygens":
            out["forms"]["huygens"] = bench_huygens(torch, max(10, args.steps // 5))
        elif f == "serve":
            out["forms"]["serve"] = bench_serve(
                torch, value, [v for v in args.serve_variants.split(",") if v] or None)
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
