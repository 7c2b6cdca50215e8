"""Python driver of the request server (sincos_server_* in include/sincos.h).

The scheduler, admission, batching and latency accounting run in C++ (one
scheduler thread per server); this module marshals arguments, replays
arrival schedules and summarizes latencies.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _capi

MODE_BATCHED, MODE_PER_REQUEST = 0, 1
EXEC_GPU, EXEC_SIM = 0, 1

COMPLETION_DTYPE = np.dtype([("id", np.int64), ("tag", np.uint64), ("status", np.int32),
                             ("batch_requests", np.int32), ("s", np.uint64), ("c", np.uint64),
                             ("n", np.int64), ("t_submit_ns", np.int64), ("t_admit_ns", np.int64),
                             ("t_launch_ns", np.int64), ("t_complete_ns", np.int64)])
assert COMPLETION_DTYPE.itemsize == ctypes.sizeof(_capi.Completion)


class _DeviceArray:
    """A device address as a float32 array (CUDA array interface)."""

    def __init__(self, ptr, n):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": "<f4",
                                         "data": (int(ptr), False), "version": 2}


class Server:
    def __init__(self, budget_bytes: int = 8 << 30, max_inflight: int = 4,
                 max_batch_requests: int = 4096, max_batch_elems: int = 0,
                 arith: int = _capi.ARITH_FUSED, method: int = _capi.METHOD_NORMALIZED,
                 mode: int = MODE_BATCHED, executor: int = EXEC_GPU, sim_batch_ns: int = 0,
                 sim_elem_ps: int = 0, sim_fail_every: int = 0, auto_release: bool = False,
                 split_elems: int = 0, stream_per_slot: bool = False):
        cfg = _capi.ServerConfig(int(budget_bytes), int(max_inflight), int(max_batch_requests),
                                 int(max_batch_elems), int(arith), int(method), int(mode),
                                 int(executor), int(sim_batch_ns), int(sim_elem_ps),
                                 int(sim_fail_every), int(bool(auto_release)), int(split_elems),
                                 int(bool(stream_per_slot)), 0)
        h = ctypes.c_void_p()
        _capi._check(_capi.lib().sincos_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.auto_release = bool(auto_release)
        self._inputs = {}  # id -> input tensor, until its completion is polled

    def submit(self, x, n=None, tag: int = 0) -> int:
        """Queue sin/cos of x; returns the id.  A tensor may still be in the
        making on the current stream: the request's batch waits on the device
        for the work queued there so far (sincos_server_submit_on), and the
        server keeps a reference to the tensor until its completion has been
        polled, so its memory cannot be reused before the batch has read it.
        An int address is taken as ready for every stream and is the
        caller's to keep alive."""
        n = int(n if n is not None else x.numel())
        rid = ctypes.c_int64()
        if isinstance(x, int):
            _capi._check(_capi.lib().sincos_server_submit(self._h, x, n, int(tag),
                                                          ctypes.byref(rid)))
            return rid.value
        import torch
        ptr = _capi._ptr(x, n)
        stream = torch.cuda.current_stream(x.device).cuda_stream
        _capi._check(_capi.lib().sincos_server_submit_on(self._h, ptr, n, int(tag), stream,
                                                         ctypes.byref(rid)))
        self._inputs[rid.value] = x
        return rid.value

    def poll(self, max_count: int = 256, timeout_s: float = 0.0):
        buf = (_capi.Completion * max_count)()
        k = ctypes.c_int32()
        _capi._check(_capi.lib().sincos_server_poll(self._h, buf, max_count, ctypes.byref(k),
                                                    int(timeout_s * 1e9)))
        out = [buf[i] for i in range(k.value)]
        for comp in out:
            self._inputs.pop(comp.id, None)  # the batch has read it
        return out

    def release(self, rid: int) -> None:
        _capi._check(_capi.lib().sincos_server_release(self._h, int(rid)))

    @staticmethod
    def outputs(comp):
        """A completed request's (s, c) as float32 tensors that alias the
        server's output buffers (no copy).  They stay valid until the request
        is released; clone them to keep the values."""
        import torch
        if comp.status != _capi.OK or not comp.s or not comp.c:
            raise ValueError("the completion carries no outputs (failed, cancelled or "
                             "auto-released)")
        return (torch.as_tensor(_DeviceArray(comp.s, comp.n), device="cuda"),
                torch.as_tensor(_DeviceArray(comp.c, comp.n), device="cuda"))

    def stats(self) -> dict:
        st = _capi.ServerStats()
        _capi._check(_capi.lib().sincos_server_stats(self._h, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in st._fields_ if name != "reserved"}

    def replay(self, xs, ns, arrival_ns) -> np.ndarray:
        """Submit request j (input address xs[j], ns[j] elements) at
        arrival_ns[j] after the start; wait for all; completions by index."""
        count = len(ns)
        if len(xs) != count or len(arrival_ns) != count:
            raise ValueError("xs, ns and arrival_ns must have the same length")
        xa = (ctypes.c_void_p * max(count, 1))(*[int(v) for v in xs])
        na = np.ascontiguousarray(ns, np.int64)
        aa = np.ascontiguousarray(arrival_ns, np.int64)
        out = np.zeros(max(count, 1), COMPLETION_DTYPE)
        rc = _capi.lib().sincos_server_replay(
            self._h, xa, na.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            aa.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), count,
            out.ctypes.data_as(ctypes.POINTER(_capi.Completion)))
        _capi._check(rc)
        return out[:count]

    def close(self) -> None:
        if self._h:
            _capi.lib().sincos_server_destroy(self._h)  # waits for batches on the device
            self._h = None
        self._inputs = {}

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def latency_summary(comp: np.ndarray) -> dict:
    """p50/p99/mean/max latency (completion - submission), in microseconds,
    and delivered throughput (elements / (last completion - first submit))."""
    lat = (comp["t_complete_ns"] - comp["t_submit_ns"]) / 1e3
    span_s = (comp["t_complete_ns"].max() - comp["t_submit_ns"].min()) / 1e9
    return {"p50_us": float(np.percentile(lat, 50)), "p99_us": float(np.percentile(lat, 99)),
            "mean_us": float(lat.mean()), "max_us": float(lat.max()),
            "requests": int(comp.size), "elements": int(comp["n"].sum()),
            "span_s": float(span_s),
            "throughput_gelem_s": float(comp["n"].sum() / span_s / 1e9) if span_s > 0 else 0.0,
            "mean_batch_requests": float(comp["batch_requests"].mean())}
