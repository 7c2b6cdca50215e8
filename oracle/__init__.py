"""CPU oracle for Mendenhall's single-precision sine-cosine pair (2004).

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The GPU product
path never imports, links or calls it, and it imports nothing from the GPU
package.

The arithmetic lives in ``sincos_oracle.c`` (plain scalar C, one element at a
time, built with contraction off).  This module only builds that file with gcc
and marshals numpy arrays through ctypes.

Arithmetic modes: ``FUSED`` (every multiply-add of the AltiVec form fused, one
rounding) and ``SPLIT`` (every product and sum rounded on its own).
Methods: ``METHOD1`` (normalized series, 2 - |p|^2 fix) and ``METHOD2``
(arctan-fit series, reciprocal of |p|^2), Sec. II of the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

FUSED, SPLIT = 0, 1
METHOD1, METHOD2 = 0, 1
VARIANT_LISTING, VARIANT_NO_FIX, VARIANT_TEXT_FIX, VARIANT_EQ2 = 0, 1, 2, 3

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sincos_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_sincos.so")

CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
          "-pthread", "-Wall", "-Wextra"]

_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle library with gcc (contraction off, no fast-math)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _f32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _f64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def lib():
    """Load the oracle library, building it first only if it is not built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build()
            L = ctypes.CDLL(_LIB)
            fp, dp = ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double)
            i64, i32, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
            c_int = ctypes.c_int
            L.oracle_reduce.restype = ctypes.c_float
            L.oracle_reduce.argtypes = [ctypes.c_float]
            L.oracle_sincos_f32.argtypes = [fp, fp, fp, i64, c_int, c_int, c_int]
            L.oracle_pair_from_reduced_f32.argtypes = [fp, fp, fp, i64, c_int, c_int, c_int, c_int]
            L.oracle_reduce_f32.argtypes = [fp, fp, i64]
            L.oracle_quarter_series.argtypes = [ctypes.c_float, c_int, c_int, fp, fp]
            L.oracle_double_angle.argtypes = [ctypes.c_float, ctypes.c_float, c_int, fp, fp]
            L.oracle_double_angle_eq2.argtypes = L.oracle_double_angle.argtypes
            L.oracle_magnitude_factor.restype = ctypes.c_float
            L.oracle_magnitude_factor.argtypes = [ctypes.c_float, ctypes.c_float, c_int, c_int]
            L.oracle_error_scan_reduced.argtypes = [u32, u32, u32, c_int, c_int, c_int, c_int,
                                                    dp, dp, dp, fp, fp,
                                                    ctypes.POINTER(ctypes.c_int64)]
            L.oracle_error_scan_variant.argtypes = L.oracle_error_scan_reduced.argtypes
            L.oracle_pair_variant.argtypes = [ctypes.c_float, c_int, c_int, c_int, fp, fp]
            L.oracle_pair_general.argtypes = [ctypes.c_float, c_int, c_int, fp, c_int, fp, c_int,
                                              c_int, fp, fp]
            L.oracle_pair_variant_f32.argtypes = [fp, fp, fp, i64, c_int, c_int, c_int, c_int]
            L.oracle_pair_general_f32.argtypes = [fp, fp, fp, i64, c_int, c_int, fp, c_int, fp,
                                                  c_int, c_int, c_int]
            L.oracle_error_scan_general.argtypes = [u32, u32, u32, c_int, c_int, fp, c_int, fp,
                                                    c_int, c_int, c_int, dp, dp, dp, fp, fp,
                                                    ctypes.POINTER(ctypes.c_int64)]
            L.oracle_sincos_backward_f32.argtypes = [fp, fp, fp, fp, fp, i64]
            L.oracle_sinusoid_forward_f32.argtypes = [fp, i64, fp, fp, fp, i32, fp, c_int, c_int,
                                                      c_int]
            L.oracle_sinusoid_adjoint_f64.argtypes = [fp, fp, i64, fp, fp, fp, i32, dp, dp, dp,
                                                      dp, dp, dp, c_int, c_int]
            L.oracle_constants.argtypes = [c_int, fp]
            L.oracle_huygens_f32.argtypes = [fp, fp, i64, fp, i32, ctypes.c_float, ctypes.c_float,
                                             fp, fp, c_int, c_int, c_int]
            L.oracle_huygens_blocks_f32.argtypes = [fp, fp, i64, fp, i32, i32, ctypes.c_float,
                                                    ctypes.c_float, fp, fp, c_int, c_int, c_int]
            _lib = L
    return _lib


def _c32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def default_threads() -> int:
    try:
        return max(1, min(len(os.sched_getaffinity(0)), 16))
    except AttributeError:  # pragma: no cover
        return max(1, min(os.cpu_count() or 1, 16))


def sincos(x, arith: int = FUSED, method: int = METHOD1, threads: int = 1):
    """Pair (s, c) of every angle in x (binary32, radians)."""
    x = _c32(x)
    s = np.empty_like(x)
    c = np.empty_like(x)
    rc = lib().oracle_sincos_f32(_f32p(x), _f32p(s), _f32p(c), x.size, arith, method, threads)
    if rc != 0:
        raise ValueError("oracle_sincos_f32 failed")
    return s, c


def pair_from_reduced(q, arith: int = FUSED, method: int = METHOD1, fixed: bool = True,
                      threads: int = 1):
    """Steps 2-4 (or 2-3 with fixed=False) on reduced angles q in [-1/2, 1/2]."""
    q = _c32(q)
    s = np.empty_like(q)
    c = np.empty_like(q)
    rc = lib().oracle_pair_from_reduced_f32(_f32p(q), _f32p(s), _f32p(c), q.size, arith, method,
                                            int(bool(fixed)), threads)
    if rc != 0:
        raise ValueError("oracle_pair_from_reduced_f32 failed")
    return s, c


def reduce(x):
    """Step 1: q1 = x/(2 pi) - nearest integer, elementwise."""
    x = _c32(x)
    q = np.empty_like(x)
    lib().oracle_reduce_f32(_f32p(x), _f32p(q), x.size)
    return q


def quarter_series(q1: float, arith: int = FUSED, method: int = METHOD1):
    s, c = ctypes.c_float(), ctypes.c_float()
    lib().oracle_quarter_series(ctypes.c_float(q1), arith, method, ctypes.byref(s),
                                ctypes.byref(c))
    return np.float32(s.value), np.float32(c.value)


def double_angle(s: float, c: float, arith: int = FUSED):
    so, co = ctypes.c_float(), ctypes.c_float()
    lib().oracle_double_angle(ctypes.c_float(s), ctypes.c_float(c), arith, ctypes.byref(so),
                              ctypes.byref(co))
    return np.float32(so.value), np.float32(co.value)


def magnitude_factor(s2: float, c2: float, arith: int = FUSED, method: int = METHOD1):
    return np.float32(lib().oracle_magnitude_factor(ctypes.c_float(s2), ctypes.c_float(c2), arith,
                                                    method))


def error_scan_reduced(bits_lo: int, bits_hi: int, stride: int = 1, arith: int = FUSED,
                       method: int = METHOD1, fixed: bool = True, threads: int | None = None):
    """Error statistics over binary32 reduced angles with bit patterns in
    [bits_lo, bits_hi] (step `stride`) against double-precision sin/cos."""
    mv, rv, ma = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    av, aa = ctypes.c_float(), ctypes.c_float()
    cnt = ctypes.c_int64()
    rc = lib().oracle_error_scan_reduced(bits_lo, bits_hi, stride, arith, method, int(fixed),
                                         threads or default_threads(), ctypes.byref(mv),
                                         ctypes.byref(rv), ctypes.byref(ma), ctypes.byref(av),
                                         ctypes.byref(aa), ctypes.byref(cnt))
    if rc != 0:
        raise ValueError("oracle_error_scan_reduced failed")
    return dict(max_vec=mv.value, rms_vec=rv.value, max_amp=ma.value, argmax_vec=av.value,
                argmax_amp=aa.value, count=cnt.value)


def error_scan_variant(bits_lo: int, bits_hi: int, stride: int = 1, arith: int = FUSED,
                       method: int = METHOD1, variant: int = VARIANT_LISTING,
                       threads: int | None = None):
    """As error_scan_reduced, for one of the Sec. II ablations (VARIANT_*)."""
    mv, rv, ma = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    av, aa = ctypes.c_float(), ctypes.c_float()
    cnt = ctypes.c_int64()
    rc = lib().oracle_error_scan_variant(bits_lo, bits_hi, stride, arith, method, variant,
                                         threads or default_threads(), ctypes.byref(mv),
                                         ctypes.byref(rv), ctypes.byref(ma), ctypes.byref(av),
                                         ctypes.byref(aa), ctypes.byref(cnt))
    if rc != 0:
        raise ValueError("oracle_error_scan_variant failed")
    return dict(max_vec=mv.value, rms_vec=rv.value, max_amp=ma.value, argmax_vec=av.value,
                argmax_amp=aa.value, count=cnt.value)


def double_angle_eq2(s: float, c: float, arith: int = FUSED):
    """One doubling with the rejected eq. (2), cos 2u = 1 - 2 sin^2 u (ablation)."""
    so, co = ctypes.c_float(), ctypes.c_float()
    lib().oracle_double_angle_eq2(ctypes.c_float(s), ctypes.c_float(c), arith, ctypes.byref(so),
                                  ctypes.byref(co))
    return np.float32(so.value), np.float32(co.value)


def pair_variant(q1: float, arith: int = FUSED, method: int = METHOD1,
                 variant: int = VARIANT_LISTING):
    s, c = ctypes.c_float(), ctypes.c_float()
    lib().oracle_pair_variant(ctypes.c_float(q1), arith, method, variant, ctypes.byref(s),
                              ctypes.byref(c))
    return np.float32(s.value), np.float32(c.value)


def pair_general(q1: float, ndoub: int, ss, cc, arith: int = FUSED, fix: bool = True):
    """The general-doubling ablation: series of len(ss), len(cc) terms for the
    angle 2 pi q1 / 2^ndoub, then ndoub eq. (1) doublings (oracle_pair_general)."""
    ss, cc = _c32(ss), _c32(cc)
    s, c = ctypes.c_float(), ctypes.c_float()
    lib().oracle_pair_general(ctypes.c_float(q1), arith, ndoub, _f32p(ss), ss.size, _f32p(cc),
                              cc.size, int(fix), ctypes.byref(s), ctypes.byref(c))
    return np.float32(s.value), np.float32(c.value)


def sincos_variant(x, arith: int = FUSED, method: int = METHOD1, variant: int = VARIANT_LISTING,
                   threads: int = 1):
    """Pairs of the angles x with one of the Sec. II ablations (pair_variant
    after the reduction of step 1)."""
    x = _c32(x)
    s = np.empty_like(x)
    c = np.empty_like(x)
    rc = lib().oracle_pair_variant_f32(_f32p(x), _f32p(s), _f32p(c), x.size, arith, method,
                                       int(variant), threads)
    if rc != 0:
        raise ValueError("oracle_pair_variant_f32 failed")
    return s, c


def sincos_general(x, ndoub: int, ss, cc, arith: int = FUSED, fix: bool = True,
                   threads: int = 1):
    """Pairs of the angles x with the general-doubling ablation (pair_general
    after the reduction of step 1)."""
    x, ss, cc = _c32(x), _c32(ss), _c32(cc)
    s = np.empty_like(x)
    c = np.empty_like(x)
    rc = lib().oracle_pair_general_f32(_f32p(x), _f32p(s), _f32p(c), x.size, arith, int(ndoub),
                                       _f32p(ss), ss.size, _f32p(cc), cc.size, int(bool(fix)),
                                       threads)
    if rc != 0:
        raise ValueError("oracle_pair_general_f32 failed")
    return s, c


def error_scan_general(bits_lo: int, bits_hi: int, ndoub: int, ss, cc, stride: int = 1,
                       arith: int = FUSED, fix: bool = True, threads: int | None = None):
    """As error_scan_reduced, for pair_general."""
    ss, cc = _c32(ss), _c32(cc)
    mv, rv, ma = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    av, aa = ctypes.c_float(), ctypes.c_float()
    cnt = ctypes.c_int64()
    rc = lib().oracle_error_scan_general(bits_lo, bits_hi, stride, arith, ndoub, _f32p(ss),
                                         ss.size, _f32p(cc), cc.size, int(fix),
                                         threads or default_threads(), ctypes.byref(mv),
                                         ctypes.byref(rv), ctypes.byref(ma), ctypes.byref(av),
                                         ctypes.byref(aa), ctypes.byref(cnt))
    if rc != 0:
        raise ValueError("oracle_error_scan_general failed")
    return dict(max_vec=mv.value, rms_vec=rv.value, max_amp=ma.value, argmax_vec=av.value,
                argmax_amp=aa.value, count=cnt.value)


def sincos_backward(s, c, gs=None, gc=None):
    """gx = gs*c - gc*s in binary32 (None counts as zero)."""
    s, c = _c32(s), _c32(c)
    gs = None if gs is None else _c32(gs)
    gc = None if gc is None else _c32(gc)
    gx = np.empty_like(s)
    lib().oracle_sincos_backward_f32(_f32p(s), _f32p(c), None if gs is None else _f32p(gs),
                                     None if gc is None else _f32p(gc), _f32p(gx), s.size)
    return gx


def sinusoid_forward(t, A, w, phi, arith: int = FUSED, method: int = METHOD1,
                     threads: int = 1):
    """y_i = sum_k A_k sin(w_k t_i + phi_k) with the method's pair, binary32."""
    t, A, w, phi = _c32(t), _c32(A), _c32(w), _c32(phi)
    y = np.empty_like(t)
    rc = lib().oracle_sinusoid_forward_f32(_f32p(t), t.size, _f32p(A), _f32p(w), _f32p(phi),
                                           A.size, _f32p(y), arith, method, threads)
    if rc != 0:
        raise ValueError("oracle_sinusoid_forward_f32 failed")
    return y


def sinusoid_adjoint(t, g, A, w, phi, arith: int = FUSED, method: int = METHOD1):
    """(gA, gw, gphi) in float64, plus the sums of |terms| per output."""
    t, g, A, w, phi = _c32(t), _c32(g), _c32(A), _c32(w), _c32(phi)
    K = A.size
    outs = [np.zeros(K, np.float64) for _ in range(6)]
    rc = lib().oracle_sinusoid_adjoint_f64(_f32p(t), _f32p(g), t.size, _f32p(A), _f32p(w),
                                           _f32p(phi), K, *[_f64p(o) for o in outs], arith,
                                           method)
    if rc != 0:
        raise ValueError("oracle_sinusoid_adjoint_f64 failed")
    gA, gw, gphi, aA, aw, aphi = outs
    return dict(gA=gA, gw=gw, gphi=gphi, abs_A=aA, abs_w=aw, abs_phi=aphi)


HUYGENS_BLOCKS = 4


def huygens(xo, yo, src, k: float, L: float, arith: int = FUSED, method: int = METHOD1,
            threads: int = 1, blocks: int = HUYGENS_BLOCKS):
    """Field (re, im) at screen points (xo, yo, L) from point sources
    src[S, 4] = (x, y, amplitude, phase); binary32.  The sources are split
    into `blocks` contiguous blocks of ceil(S / blocks), each summed in source
    order, and the block sums are added in block order (blocks=1: the plain
    sum in source order)."""
    xo, yo = _c32(xo), _c32(yo)
    src = np.ascontiguousarray(src, np.float32).reshape(-1, 4)
    re = np.empty_like(xo)
    im = np.empty_like(xo)
    rc = lib().oracle_huygens_blocks_f32(_f32p(xo), _f32p(yo), xo.size, _f32p(src),
                                         src.shape[0], int(blocks), np.float32(k), np.float32(L),
                                         _f32p(re), _f32p(im), arith, method, threads)
    if rc != 0:
        raise ValueError("oracle_huygens_blocks_f32 failed")
    return re, im


def constants(method: int = METHOD1):
    out = np.zeros(8, np.float32)
    lib().oracle_constants(method, _f32p(out))
    return out
