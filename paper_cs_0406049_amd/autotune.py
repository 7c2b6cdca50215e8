"""Launch-shape autotuner for the ragged form.

For a ragged batch it times one plan per candidate (block, unroll, grid, lds) with
HIP events (the kernel only, each candidate replayed a few times after a
warm-up), then re-times the fastest few in interleaved rounds (so that a slow
spell of the GPU hits every finalist alike) and keeps the one with the lowest
median.  The choice is cached in a JSON file keyed by
device architecture, CU count and a bucket of the batch's size (segment count
and total elements, each rounded to a power of two), so a later batch of a
similar size reuses it without timing.

    shape = autotune.tune_ragged(segs, lens)        # (block, unroll, grid, lds)
    plan = _capi.RaggedPlan(segs, lens, launch=shape)

or, with install_default=True, the choice becomes the library's process-wide default
for ragged calls that pass no launch shape (sincos_set_tuning).
"""
from __future__ import annotations

import json
import math
import os
import threading

from . import _capi

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mi355_sincos", "tune.json")

BLOCKS = (64, 128, 256, 512)
UNROLLS = (1, 2, 4)
# resident waves per CU for a persistent grid (grid = CUs * waves / (block / 64));
# 0 = one workgroup per unit of work (no persistence)
WAVES_PER_CU = (8, 16, 32, 64, 128, 0)
COVER = 1 << 30  # a grid this large is capped to the number of units
# For the one-workgroup-per-unit grid: caps on resident waves per CU, applied
# by reserving LDS in each workgroup (0 = no cap).  Fewer tiles in flight
# keep fewer DRAM rows open; too few starve the reads.
WAVE_CAPS = (0, 24, 16)
LDS_PER_CU = 160 * 1024
MAX_LDS = 65536

_lock = threading.Lock()


def _bucket(v: int) -> int:
    return 0 if v <= 0 else 1 << int(math.ceil(math.log2(v)))


def cache_key(arch: str, cus: int, count: int, elements: int, arith: int, method: int) -> str:
    return "%s/cu%d/ragged/a%d-m%d/seg%d/el%d" % (arch, cus, arith, method, _bucket(count),
                                                 _bucket(elements))


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = DEFAULT_CACHE) -> None:
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lds_for_cap(block: int, cap: int):
    """LDS bytes per workgroup that hold a CU to about `cap` resident waves
    (-1: reserve none; None: not expressible for this block size)."""
    if cap == 0:
        return -1
    wgs = cap // (block // 64)
    if wgs < 1:
        return None
    lds = (LDS_PER_CU // wgs) // 256 * 256
    return lds if lds <= MAX_LDS else None


def candidates(cus: int):
    """(block, unroll, grid, lds) launch shapes to time; lds -1 = none."""
    for block in BLOCKS:
        for unroll in UNROLLS:
            for wpc in WAVES_PER_CU:
                if wpc:
                    yield (block, unroll, max(1, cus * wpc * 64 // block), -1)
                    continue
                for cap in WAVE_CAPS:
                    lds = lds_for_cap(block, cap)
                    if lds is not None:
                        yield (block, unroll, COVER, lds)


def time_plan(torch, plan, reps: int = 5) -> float:
    """Average milliseconds of one plan launch (kernel only)."""
    plan.launch()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    st = torch.cuda.current_stream()
    a.record(st)
    for _ in range(reps):
        plan.launch()
    b.record(st)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def install(form: str, shape) -> None:
    """Make shape = (block, unroll, grid[, lds]) the library's default launch
    shape for form ("plain" or "ragged"), keeping the other form's default
    (lds -1, no reservation, is installed as 0)."""
    if form not in ("plain", "ragged"):
        raise ValueError("form must be 'plain' or 'ragged'")
    cur = _capi.get_tuning()
    sh = dict(zip(("block", "unroll", "grid", "lds"), (int(v) for v in shape)))
    sh.setdefault("lds", 0)
    sh["lds"] = max(sh["lds"], 0)
    cur[form] = sh
    _capi.set_tuning(cur)


FINALISTS = 6
ROUNDS = 5


def tune_ragged(segs, lens=None, arith: int = _capi.ARITH_FUSED,
                method: int = _capi.METHOD_NORMALIZED, cache_path: str | None = DEFAULT_CACHE,
                force: bool = False, reps: int = 5, verbose: bool = False,
                install_default: bool = False, finalists: int = FINALISTS,
                rounds: int = ROUNDS):
    """Best (block, unroll, grid, lds) for this batch (from the cache if present).
    The arrays' contents are overwritten with valid outputs while timing.
    With install_default, the choice also becomes the library's default for
    ragged calls (grid capped there to each call's units)."""
    best, _ = _tune_ragged(segs, lens, arith, method, cache_path, force, reps, verbose,
                           finalists, rounds)
    if install_default:
        install("ragged", best)
    return best


def tune_ragged_table(segs, lens=None, arith: int = _capi.ARITH_FUSED,
                      method: int = _capi.METHOD_NORMALIZED, reps: int = 5,
                      verbose: bool = False, finalists: int = FINALISTS,
                      rounds: int = ROUNDS):
    """Time every candidate (no cache) and return (best, [(ms, shape), ...]):
    the finalists first, fastest median first (their ms is that median), then
    the other candidates fastest first (their ms is the single first pass)."""
    return _tune_ragged(segs, lens, arith, method, None, True, reps, verbose, finalists, rounds)


def _tune_ragged(segs, lens, arith, method, cache_path, force, reps, verbose, finalists=FINALISTS,
                 rounds=ROUNDS):
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    arch = getattr(props, "gcnArchName", "unknown").split(":")[0]
    cus = props.multi_processor_count
    if lens is None:
        lens = [int(x.numel()) for x, _, _ in segs]
    key = cache_key(arch, cus, len(lens), int(sum(lens)), arith, method)
    with _lock:
        cache = load_cache(cache_path) if cache_path else {}
        if not force and key in cache:
            return tuple(cache[key]["shape"]), []
    results = []
    for shape in candidates(cus):
        plan = _capi.RaggedPlan(segs, lens, arith, method, launch=shape)
        ms = time_plan(torch, plan, reps)
        plan.destroy()
        results.append((ms, shape))
        if verbose:
            print("autotune %-18s %.4f ms" % (shape, ms), flush=True)
    results.sort()
    # second stage: the fastest few again, in interleaved rounds
    k = max(1, min(finalists, len(results)))
    plans = [(shape, _capi.RaggedPlan(segs, lens, arith, method, launch=shape))
             for _, shape in results[:k]]
    times = {shape: [] for shape, _ in plans}
    try:
        for r in range(max(1, rounds)):
            for j in range(k):
                shape, plan = plans[(j + r) % k]
                times[shape].append(time_plan(torch, plan, reps))
    finally:
        for _, plan in plans:
            plan.destroy()
    final = sorted((sorted(v)[len(v) // 2], shape) for shape, v in times.items())
    if verbose:
        for ms, shape in final:
            print("autotune finalist %-18s median %.4f ms" % (shape, ms), flush=True)
    results = final + results[k:]
    best_ms, best = results[0]
    if cache_path:
        with _lock:
            cache = load_cache(cache_path)
            cache[key] = {"shape": list(best), "ms": best_ms, "elements": int(sum(lens)),
                          "segments": len(lens), "tried": len(results)}
            save_cache(cache, cache_path)
    return best, results
