"""ctypes binding of libmi355_sincos.so (declared in include/sincos.h).

Argument marshalling only: every step of the computation runs in the HIP
library.  Array arguments may be torch tensors (float32, contiguous, on the
GPU) or raw device addresses (int).  `stream` defaults to torch's current HIP
stream.  A non-OK status raises SincosError with the library's message.
If the shared library has not been built, loading it raises RuntimeError:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import json
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmi355_sincos.so")

OK, EINVAL, EOVERLAP, ENOMEM, EHIP, ENODEV, ECANCELED, EBUDGET = 0, -1, -2, -3, -4, -5, -6, -7
ARITH_FUSED, ARITH_SPLIT, ARITH_CONTRACT = 0, 1, 2
METHOD_NORMALIZED, METHOD_ARCTAN = 0, 1
VARIANT_LISTING, VARIANT_NO_FIX, VARIANT_TEXT_FIX, VARIANT_EQ2 = 0, 1, 2, 3
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "EOVERLAP", -3: "ENOMEM", -4: "EHIP", -5: "ENODEV",
                -6: "ECANCELED", -7: "EBUDGET"}


class SincosError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, message))
        self.status = status
        self.message = message


class Launch(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("lds", ctypes.c_int32)]


class Seg(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("s", ctypes.c_void_p), ("c", ctypes.c_void_p)]


class ServerConfig(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_inflight", ctypes.c_int32),
                ("max_batch_requests", ctypes.c_int32), ("max_batch_elems", ctypes.c_int64),
                ("arith", ctypes.c_int32), ("method", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("executor", ctypes.c_int32), ("sim_batch_ns", ctypes.c_int64),
                ("sim_elem_ps", ctypes.c_int64), ("sim_fail_every", ctypes.c_int32),
                ("auto_release", ctypes.c_int32), ("split_elems", ctypes.c_int64),
                ("stream_per_slot", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("tag", ctypes.c_uint64), ("status", ctypes.c_int32),
                ("batch_requests", ctypes.c_int32), ("s", ctypes.c_void_p),
                ("c", ctypes.c_void_p), ("n", ctypes.c_int64), ("t_submit_ns", ctypes.c_int64),
                ("t_admit_ns", ctypes.c_int64), ("t_launch_ns", ctypes.c_int64),
                ("t_complete_ns", ctypes.c_int64)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("elements_completed", ctypes.c_int64),
                ("budget_in_use", ctypes.c_int64), ("budget_peak", ctypes.c_int64),
                ("inflight_peak", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_lock = threading.Lock()
_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32

_SIGNATURES = {
    "sincos_f32": (ctypes.c_int, [_P, _P, _P, _I64, _P]),
    "sincos_f32_ex": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _I32, ctypes.POINTER(Launch), _P]),
    "sincos_f32_ragged": (ctypes.c_int, [ctypes.POINTER(Seg), ctypes.POINTER(_I64), _I32, _P]),
    "sincos_f32_ragged_ex": (ctypes.c_int, [ctypes.POINTER(Seg), ctypes.POINTER(_I64), _I32, _I32,
                                            _I32, ctypes.POINTER(Launch), _P]),
    "sincos_ragged_plan_create": (ctypes.c_int, [ctypes.POINTER(Seg), ctypes.POINTER(_I64), _I32,
                                                 _I32, _I32, ctypes.POINTER(Launch),
                                                 ctypes.POINTER(_P)]),
    "sincos_ragged_plan_launch": (ctypes.c_int, [_P, _P]),
    "sincos_ragged_plan_graph_launch": (ctypes.c_int, [_P, _P]),
    "sincos_ragged_plan_info": (ctypes.c_int, [_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32),
                                               ctypes.POINTER(_I32), ctypes.POINTER(_I64),
                                               ctypes.POINTER(_I64)]),
    "sincos_ragged_plan_destroy": (ctypes.c_int, [_P]),
    "sincos_f32_backward": (ctypes.c_int, [_P, _P, _P, _P, _P, _I64, _P]),
    "sinusoid_f32_forward": (ctypes.c_int, [_P, _I64, _P, _P, _P, _I32, _P, _P]),
    "sinusoid_f32_backward_workspace_bytes": (ctypes.c_int64, [_I64, _I32]),
    "sinusoid_f32_residual_workspace_bytes": (ctypes.c_int64, [_I64]),
    "sinusoid_f32_residual": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _I32, _P, _P, _P, _I64,
                                             _P]),
    "sinusoid_f32_backward": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _I32, _P, _P, _P, _P, _I64,
                                             _P]),
    "sinusoid_f32_fit_step_workspace_bytes": (_I64, [_I64, _I32]),
    "sinusoid_f32_fit_step": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _I32, _P, _P, _P, _P, _P,
                                             _I64, _P]),
    "sinusoid_f32_fit_step_noalloc": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _I32, _P, _P, _P,
                                                     _P, _P]),
    "sincos_copy_ceiling_f32": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.POINTER(Launch), _P]),
    "sincos_stream_probe_f32": (ctypes.c_int, [_I32, _I32, _P, _P, _P, _I64,
                                               ctypes.POINTER(Launch), _P]),
    "sincos_f32_interleaved": (ctypes.c_int, [_P, _P, _I64, _I32, _P]),
    "sincos_pair_ceiling_f32": (ctypes.c_int, [_P, _P, _I64, _I32, _P]),
    "sincos_f32_variant": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _I32, _I32, _P]),
    "sincos_f32_doublings": (ctypes.c_int, [_P, _P, _P, _I64, _I32, _I32,
                                            ctypes.POINTER(ctypes.c_float), _I32,
                                            ctypes.POINTER(ctypes.c_float), _I32, _I32, _P]),
    "huygens_f32": (ctypes.c_int, [_P, _P, _I64, _P, _I32, ctypes.c_float, ctypes.c_float, _P, _P,
                                   _P]),
    "huygens_term_ceiling_f32": (ctypes.c_int, [_P, _P, _I64, _P, _I32, ctypes.c_float,
                                                ctypes.c_float, _P, _P, _P]),
    "sincos_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(_P)]),
    "sincos_server_submit": (ctypes.c_int, [_P, _P, _I64, ctypes.c_uint64, ctypes.POINTER(_I64)]),
    "sincos_server_submit_on": (ctypes.c_int, [_P, _P, _I64, ctypes.c_uint64, _P,
                                               ctypes.POINTER(_I64)]),
    "sincos_server_poll": (ctypes.c_int, [_P, ctypes.POINTER(Completion), _I32,
                                          ctypes.POINTER(_I32), _I64]),
    "sincos_server_release": (ctypes.c_int, [_P, _I64]),
    "sincos_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(ServerStats)]),
    "sincos_server_replay": (ctypes.c_int, [_P, ctypes.POINTER(_P), ctypes.POINTER(_I64),
                                            ctypes.POINTER(_I64), _I32,
                                            ctypes.POINTER(Completion)]),
    "sincos_server_destroy": (ctypes.c_int, [_P]),
    "sincos_set_tuning": (ctypes.c_int, [ctypes.c_char_p]),
    "sincos_get_tuning": (ctypes.c_int64, [ctypes.c_char_p, _I64]),
    "sincos_last_error": (ctypes.c_char_p, []),
    "sincos_version": (ctypes.c_char_p, []),
}


def lib():
    """The loaded library (raises RuntimeError if it is not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(
                    "libmi355_sincos.so is not built (python -m paper_cs_0406049_amd.build); "
                    "this package has no CPU or fallback path")
            # PyTorch-ROCm ships its own HIP runtime under the same soname.  Load
            # torch first so the library binds to that one runtime: device
            # pointers and streams from torch are then valid here.
            try:
                import torch  # noqa: F401
            except ImportError:
                pass
            L = ctypes.CDLL(LIB_PATH)
            for name, (res, args) in _SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


def last_error() -> str:
    return lib().sincos_last_error().decode()


def _check(status: int) -> int:
    if status != OK:
        raise SincosError(status, last_error())
    return status


def _ptr(a, need=None):
    """Device address of a tensor (float32, contiguous, on the GPU) or an int.
    A tensor must hold at least `need` elements when that is given (a raw
    address is taken as is)."""
    if a is None:
        return None
    if isinstance(a, int):
        return a
    if not a.is_cuda:
        raise ValueError("array must be on the GPU")
    if a.dtype.itemsize != 4 or not a.is_floating_point():
        raise ValueError("array must be float32")
    if not a.is_contiguous():
        raise ValueError("array must be contiguous")
    if need is not None and a.numel() < need:
        raise ValueError("array holds %d elements, the call needs %d" % (a.numel(), need))
    return a.data_ptr()


def _raw_ptr(a, need_bytes=None):
    """Device address of a contiguous tensor of any dtype, an int, or None."""
    if a is None or isinstance(a, int):
        return a
    if not a.is_cuda:
        raise ValueError("array must be on the GPU")
    if not a.is_contiguous():
        raise ValueError("array must be contiguous")
    if need_bytes is not None and a.numel() * a.element_size() < need_bytes:
        raise ValueError("array holds %d bytes, the call needs %d"
                         % (a.numel() * a.element_size(), need_bytes))
    return a.data_ptr()


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _launch(launch):
    if launch is None:
        return None
    if isinstance(launch, Launch):
        return ctypes.byref(launch)
    b, u, g, r = (tuple(launch) + (0, 0, 0, 0))[:4]
    return ctypes.byref(Launch(int(b), int(u), int(g), int(r)))


def _numel(a, n):
    if n is not None:
        return int(n)
    return int(a.numel())


# ---------------------------------------------------------------------------
# Entry points, same names as the C ABI.


def sincos_f32(x, s, c, n=None, stream=None) -> None:
    n = _numel(x, n)
    _check(lib().sincos_f32(_ptr(x, n), _ptr(s, n), _ptr(c, n), n, _stream(stream)))


def sincos_f32_ex(x, s, c, n=None, arith=ARITH_FUSED, method=METHOD_NORMALIZED, launch=None,
                  stream=None) -> None:
    n = _numel(x, n)
    _check(lib().sincos_f32_ex(_ptr(x, n), _ptr(s, n), _ptr(c, n), n, int(arith), int(method),
                               _launch(launch), _stream(stream)))


def sincos_f32_interleaved(x, out, n=None, layout=0, stream=None) -> None:
    """layout 0: complex64 (cos, sin) pairs; 1: blocks of 4 sines, 4 cosines."""
    n = _numel(x, n)
    out_floats = 2 * n if int(layout) == 0 else 8 * ((n + 3) // 4)
    _check(lib().sincos_f32_interleaved(_ptr(x, n), _raw_ptr(out, 4 * out_floats), n, int(layout),
                                        _stream(stream)))


def sincos_copy_ceiling_f32(x, s, c, n=None, launch=None, stream=None) -> None:
    n = _numel(x, n)
    _check(lib().sincos_copy_ceiling_f32(_ptr(x, n), _ptr(s, n), _ptr(c, n), n,
                                         _launch(launch), _stream(stream)))


PROBE_READ, PROBE_WRITE, PROBE_WRITE1, PROBE_COPY, PROBE_COPY_BATCH, PROBE_COPY_SPLIT, \
    PROBE_COPY_LDS, PROBE_COPY_XCD = range(8)
PROBE_NAMES = {PROBE_READ: "read", PROBE_WRITE: "write", PROBE_WRITE1: "write1",
               PROBE_COPY: "copy", PROBE_COPY_BATCH: "copy_batch",
               PROBE_COPY_SPLIT: "copy_split", PROBE_COPY_LDS: "copy_lds",
               PROBE_COPY_XCD: "copy_xcd"}
# bytes moved per element by each probe
PROBE_BYTES = {PROBE_READ: 4, PROBE_WRITE: 8, PROBE_WRITE1: 4, PROBE_COPY: 12,
               PROBE_COPY_BATCH: 12, PROBE_COPY_SPLIT: 12, PROBE_COPY_LDS: 12, PROBE_COPY_XCD: 12}


def sincos_stream_probe_f32(probe, x, s, c, n, launch=None, policy=-1, stream=None) -> None:
    """A memory-traffic probe (PROBE_*) over n elements; x or c may be None
    where the probe does not use them.  policy -1: the plain kernel's."""
    n = int(n)
    ns = 1 if probe == PROBE_READ else n
    _check(lib().sincos_stream_probe_f32(int(probe), int(policy), _ptr(x, n), _ptr(s, ns),
                                         _ptr(c, n), n, _launch(launch), _stream(stream)))


def sincos_pair_ceiling_f32(x, out, n=None, reps=1, stream=None) -> None:
    n = _numel(x, n)
    _check(lib().sincos_pair_ceiling_f32(_ptr(x, n), _ptr(out, n), n, int(reps),
                                         _stream(stream)))


def sincos_f32_variant(x, s, c, n=None, arith=ARITH_FUSED, method=METHOD_NORMALIZED,
                       variant=VARIANT_LISTING, stream=None) -> None:
    """One of the Sec. II ablations of the method (VARIANT_*)."""
    n = _numel(x, n)
    _check(lib().sincos_f32_variant(_ptr(x, n), _ptr(s, n), _ptr(c, n), n, int(arith),
                                    int(method), int(variant), _stream(stream)))


def sincos_f32_doublings(x, s, c, ndoub, ss, cc, n=None, arith=ARITH_FUSED, fix=True,
                         stream=None) -> None:
    """The general ablation: series ss, cc (host sequences of binary32
    coefficients) for 2 pi q / 2^ndoub, then ndoub doublings."""
    n = _numel(x, n)
    ssa = (ctypes.c_float * max(len(ss), 1))(*[float(v) for v in ss])
    cca = (ctypes.c_float * max(len(cc), 1))(*[float(v) for v in cc])
    _check(lib().sincos_f32_doublings(_ptr(x, n), _ptr(s, n), _ptr(c, n), n, int(arith),
                                      int(ndoub), ssa, len(ss), cca, len(cc), int(bool(fix)),
                                      _stream(stream)))


def _seg_tables(segs, lens):
    """Segment and length tables as contiguous arrays (no per-segment ctypes
    objects, so large batches marshal quickly)."""
    import numpy as np
    count = len(segs)
    tab = np.zeros((max(count, 1), 3), np.uint64)
    if lens is None:
        lt = np.array([int(x.numel()) for x, _, _ in segs] or [0], np.int64)
    else:
        lt = np.ascontiguousarray(lens, np.int64) if count else np.zeros(1, np.int64)
        if lt.shape != (count,) and count:
            raise ValueError("lens must hold one length per segment")
    if count:
        tab[:count] = [[_ptr(x, n) or 0, _ptr(s, n) or 0, _ptr(c, n) or 0]
                       for (x, s, c), n in zip(segs, lt[:count].tolist())]
    st = tab.ctypes.data_as(ctypes.POINTER(Seg))
    lp = lt.ctypes.data_as(ctypes.POINTER(_I64))
    return (st, tab), (lp, lt), count


class SegTable:
    """The pointer and length tables of a ragged batch, marshalled once.

    SegTable(segs, lens) checks each (x, s, c) tensor and reads its address
    (about 0.4 us per tensor in Python, 5 ms for 4096 segments); a one-shot
    sincos_f32_ragged(table) then passes the ready tables to the library
    with no per-segment Python work.  The table keeps its tensors alive.
    SegTable.from_pointers(ptrs, lens) wraps device addresses the caller
    already holds: ptrs is a (count, 3) array of uint64 (x, s, c), lens a
    (count,) array of int64; the caller keeps that memory alive.  The
    library validates every call's tables (sizes, alignment, overlaps)."""

    def __init__(self, segs=None, lens=None):
        if segs is None:
            return
        (st, tab), (lp, lt), count = _seg_tables(segs, lens)
        self._st, self._tab, self._lp, self._lt, self.count = st, tab, lp, lt, count
        self._keep = list(segs)

    @classmethod
    def from_pointers(cls, ptrs, lens):
        import numpy as np
        tab = np.ascontiguousarray(ptrs, np.uint64)
        lt = np.ascontiguousarray(lens, np.int64)
        count = int(lt.shape[0]) if lt.ndim == 1 else -1
        if lt.ndim != 1 or tab.shape != (count, 3):
            raise ValueError("ptrs must be (count, 3) and lens (count,)")
        if count == 0:
            tab, lt = np.zeros((1, 3), np.uint64), np.zeros(1, np.int64)
        self = cls()
        self._tab, self._lt, self.count, self._keep = tab, lt, count, []
        self._st = tab.ctypes.data_as(ctypes.POINTER(Seg))
        self._lp = lt.ctypes.data_as(ctypes.POINTER(_I64))
        return self


def sincos_f32_ragged(segs, lens=None, stream=None, arith=ARITH_FUSED, method=METHOD_NORMALIZED,
                      launch=None) -> None:
    """segs: sequence of (x, s, c), lens: lengths (default: x.numel()); or a
    SegTable built beforehand (lens must then be None)."""
    if isinstance(segs, SegTable):
        if lens is not None:
            raise ValueError("a SegTable carries its own lengths")
        st, lt, count = segs._st, segs._lp, segs.count
    else:
        (st, _keep1), (lt, _keep2), count = _seg_tables(segs, lens)
    _check(lib().sincos_f32_ragged_ex(st, lt, count, int(arith), int(method), _launch(launch),
                                      _stream(stream)))


class RaggedPlan:
    """A ragged batch validated and uploaded once; launch() or graph_launch()
    then enqueue a single kernel (or its graph) with no host work."""

    def __init__(self, segs, lens=None, arith=ARITH_FUSED, method=METHOD_NORMALIZED,
                 launch=None):
        (st, _keep1), (lt, _keep2), count = _seg_tables(segs, lens)
        h = _P()
        _check(lib().sincos_ragged_plan_create(st, lt, count, int(arith), int(method),
                                               _launch(launch), ctypes.byref(h)))
        self._h = h
        self._keep = list(segs)  # the plan holds raw pointers: keep the arrays alive

    def launch(self, stream=None):
        _check(lib().sincos_ragged_plan_launch(self._h, _stream(stream)))

    def graph_launch(self, stream=None):
        _check(lib().sincos_ragged_plan_graph_launch(self._h, _stream(stream)))

    def info(self):
        b, u, g = _I32(), _I32(), _I32()
        units, elems = _I64(), _I64()
        _check(lib().sincos_ragged_plan_info(self._h, ctypes.byref(b), ctypes.byref(u),
                                             ctypes.byref(g), ctypes.byref(units),
                                             ctypes.byref(elems)))
        return dict(block=b.value, unroll=u.value, grid=g.value, units=units.value,
                    elements=elems.value)

    def destroy(self):
        if self._h:
            lib().sincos_ragged_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass


def sincos_f32_backward(s, c, gs, gc, gx, n=None, stream=None) -> None:
    n = _numel(s, n)
    _check(lib().sincos_f32_backward(_ptr(s, n), _ptr(c, n), _ptr(gs, n), _ptr(gc, n),
                                     _ptr(gx, n), n, _stream(stream)))


def sinusoid_f32_forward(t, A, w, phi, y, N=None, K=None, stream=None) -> None:
    N, K = _numel(t, N), _numel(A, K)
    _check(lib().sinusoid_f32_forward(_ptr(t, N), N, _ptr(A, K), _ptr(w, K), _ptr(phi, K), K,
                                      _ptr(y, N), _stream(stream)))


def sinusoid_f32_residual_workspace_bytes(N: int) -> int:
    return int(lib().sinusoid_f32_residual_workspace_bytes(int(N)))


def sinusoid_f32_residual(t, y_obs, A, w, phi, r, loss, workspace, workspace_bytes=None, N=None,
                          K=None, stream=None) -> None:
    """r = model(t) - y_obs and loss[0] = 1/2 sum r^2 (deterministic order)."""
    N, K = _numel(t, N), _numel(A, K)
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().sinusoid_f32_residual(_ptr(t, N), _ptr(y_obs, N), N, _ptr(A, K), _ptr(w, K),
                                       _ptr(phi, K), K, _ptr(r, N), _ptr(loss, 1),
                                       _raw_ptr(workspace, int(workspace_bytes)),
                                       int(workspace_bytes), _stream(stream)))


def sinusoid_f32_backward_workspace_bytes(N: int, K: int) -> int:
    return int(lib().sinusoid_f32_backward_workspace_bytes(int(N), int(K)))


def sinusoid_f32_backward(t, g, A, w, phi, gA, gw, gphi, workspace, workspace_bytes=None,
                          N=None, K=None, stream=None) -> None:
    N = _numel(t, N)
    K = _numel(A, K)
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().sinusoid_f32_backward(_ptr(t, N), _ptr(g, N), N, _ptr(A, K), _ptr(w, K),
                                       _ptr(phi, K), K, _ptr(gA, K), _ptr(gw, K), _ptr(gphi, K),
                                       _raw_ptr(workspace, int(workspace_bytes)),
                                       int(workspace_bytes), _stream(stream)))


def sinusoid_f32_fit_step_workspace_bytes(N: int, K: int) -> int:
    return int(lib().sinusoid_f32_fit_step_workspace_bytes(int(N), int(K)))


def sinusoid_f32_fit_step(t, y_obs, A, w, phi, loss, gA, gw, gphi, workspace,
                          workspace_bytes=None, N=None, K=None, stream=None) -> None:
    """loss[0] = 1/2 sum (y - y_obs)^2 and its gradients in one pass."""
    N = _numel(t, N)
    K = _numel(A, K)
    if workspace_bytes is None:
        workspace_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
    _check(lib().sinusoid_f32_fit_step(_ptr(t, N), _ptr(y_obs, N), N, _ptr(A, K), _ptr(w, K),
                                       _ptr(phi, K), K, _ptr(loss, 1), _ptr(gA, K), _ptr(gw, K),
                                       _ptr(gphi, K), _raw_ptr(workspace, int(workspace_bytes)),
                                       int(workspace_bytes), _stream(stream)))


# Bytes of the library's static scratch used by sinusoid_f32_fit_step_noalloc
# (SINCOS_FIT_SCRATCH_BYTES in sincos.h).
FIT_SCRATCH_BYTES = 8 << 20


def sinusoid_f32_fit_step_noalloc(t, y_obs, A, w, phi, loss, gA, gw, gphi, N=None, K=None,
                                  stream=None) -> None:
    """sinusoid_f32_fit_step with its partials in the library's static scratch
    (no device allocation); calls on one GPU must not overlap in time."""
    N = _numel(t, N)
    K = _numel(A, K)
    _check(lib().sinusoid_f32_fit_step_noalloc(_ptr(t, N), _ptr(y_obs, N), N, _ptr(A, K),
                                               _ptr(w, K), _ptr(phi, K), K, _ptr(loss, 1),
                                               _ptr(gA, K), _ptr(gw, K), _ptr(gphi, K),
                                               _stream(stream)))


def huygens_f32(xo, yo, src, k, L, re, im, P=None, S=None, stream=None) -> None:
    """src: [S, 4] float32 (x, y, amplitude, phase), 16-byte aligned."""
    P = _numel(xo, P)
    S = int(S if S is not None else src.numel() // 4)
    _check(lib().huygens_f32(_ptr(xo, P), _ptr(yo, P), P, _ptr(src, 4 * S), S, float(k),
                             float(L), _ptr(re, P), _ptr(im, P), _stream(stream)))


def huygens_term_ceiling_f32(xo, yo, src8, reps, k, L, re, im, P=None, stream=None) -> None:
    """huygens_f32 over the 8 sources of src8 repeated reps times, the
    sources held in registers (the term's ceiling)."""
    P = _numel(xo, P)
    _check(lib().huygens_term_ceiling_f32(_ptr(xo, P), _ptr(yo, P), P, _ptr(src8, 32), int(reps),
                                          float(k), float(L), _ptr(re, P), _ptr(im, P),
                                          _stream(stream)))


def set_tuning(shapes) -> None:
    """Install process-wide default launch shapes.  shapes: None (built-in
    defaults) or {"plain": {...}, "ragged": {...}} with any of the integer
    fields "block", "unroll", "grid", "lds"; a (block, unroll, grid[, lds])
    tuple may stand for a form's dict."""
    if shapes is None:
        _check(lib().sincos_set_tuning(None))
        return
    doc = {}
    for form, sh in shapes.items():
        if isinstance(sh, (tuple, list)):
            sh = dict(zip(("block", "unroll", "grid", "lds"), sh))
        doc[form] = {k: int(v) for k, v in sh.items()}
    _check(lib().sincos_set_tuning(json.dumps(doc).encode()))


def get_tuning() -> dict:
    """The default launch shapes in effect, as {"plain": {...}, "ragged": {...}}."""
    n = lib().sincos_get_tuning(None, 0)
    buf = ctypes.create_string_buffer(int(n) + 1)
    lib().sincos_get_tuning(buf, n + 1)
    return json.loads(buf.value.decode())


def version() -> str:
    return lib().sincos_version().decode()
