"""The pins catch plausible mistakes.

Each case plants one mistake in a copy of the oracle's C source (on the CPU,
in a temporary directory), builds it with the oracle's own flags, and runs a
fast subset of the pins of test_oracle_pins.py against it.  The unmodified
source must pass every pin; every mutant must fail at least one.
"""
import ctypes
import math
import os
import subprocess

import numpy as np
import pytest

from golden import loader

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle",
                   "sincos_oracle.c")

MUTANTS = {
    "ss2_sign": ("k.ss2 = (float)-0.645963615;", "k.ss2 = (float)0.645963615;"),
    "drop_ss4": ("float t = mul_add(q2, k.ss4, k.ss3, arith);", "float t = k.ss3;"),
    "drop_cc3": ("float u = mul_add(q2, k.cc3, k.cc2, arith);", "float u = k.cc2;"),
    "cc1_cc2_swapped": ("u = mul_add(q2, u, k.cc1, arith);\n    *c1 = mul_add(q2, u, 1.0f, arith);",
                        "u = mul_add(q2, u, k.cc2, arith);\n    *c1 = mul_add(q2, u, 1.0f, arith);"),
    "ss3_digit_typo": ("k.ss3 = (float)0.0796819754;", "k.ss3 = (float)0.0769819754;"),
    "doubling_plus": ("*c_out = mul_sub_from(s, s, cc, arith);", "*c_out = mul_add(s, s, cc, arith);"),
    "doubling_no_two": ("*s_out = 2.0f * sc;", "*s_out = sc;"),
    "rejected_doubling": ("*c_out = mul_sub_from(s, s, cc, arith);",
                          "(void)cc; *c_out = mul_sub_from(2.0f * s, s, 1.0f, arith);"),
    "one_doubling": ("oracle_double_angle(s2, c2, arith, &s3, &c3);", "s3 = s2; c3 = c2;"),
    "no_fix": ("*s = s3 * m;\n    *c = c3 * m;", "(void)m;\n    *s = s3;\n    *c = c3;"),
    "fix_sign": ("return mul_sub_from(s2, s2, inner, arith);", "return mul_add(s2, s2, inner, arith);"),
    "ties_away": ("float r = rintf(x1);", "float r = roundf(x1);"),
    "truncate": ("float r = rintf(x1);", "float r = truncf(x1);"),
    "reduce_sign": ("return x1 - r;", "return r - x1;"),
    "pi_digits": ("(float)(1.0 / (2.0 * 3.1415926536))", "(float)(1.0 / (2.0 * 3.14159))"),
    "split_fuses": ("float p = a * b;\n    return p + c;", "return fmaf(a, b, c);"),
    "fused_splits": ("return fmaf(a, b, c);\n    float p = a * b;\n    return p + c;",
                     "{ float p = a * b; return p + c; }"),
    "flush_subnormal": ("float x1 = x * reduction_constant();",
                        "float x1 = x * reduction_constant();\n    if (fabsf(x1) < 1.17549435e-38f) x1 = 0.0f;"),
    "fix_before_doubling": ("*s = s3 * m;\n    *c = c3 * m;",
                            "oracle_double_angle(s2 * m, c2 * m, arith, s, c);"),
}

FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared", "-pthread"]


def _build(tmp_path, name, src):
    c = tmp_path / (name + ".c")
    so = tmp_path / ("lib" + name + ".so")
    c.write_text(src)
    subprocess.check_call(["gcc", *FLAGS, str(c), "-o", str(so), "-lm"])
    L = ctypes.CDLL(str(so))
    fp = ctypes.POINTER(ctypes.c_float)
    dp = ctypes.POINTER(ctypes.c_double)
    L.oracle_sincos_f32.argtypes = [fp, fp, fp, ctypes.c_int64, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.oracle_reduce_f32.argtypes = [fp, fp, ctypes.c_int64]
    L.oracle_error_scan_reduced.argtypes = [ctypes.c_uint32] * 3 + [ctypes.c_int] * 4 + [
        dp, dp, dp, fp, fp, ctypes.POINTER(ctypes.c_int64)]
    L.oracle_constants.argtypes = [ctypes.c_int, fp]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def _sincos(L, x, arith, method=0):
    x = np.ascontiguousarray(x, np.float32)
    s, c = np.empty_like(x), np.empty_like(x)
    L.oracle_sincos_f32(_p(x), _p(s), _p(c), x.size, arith, method, 1)
    return s, c


def _scan(L, arith, stride):
    mv, rv, ma = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    a, b, n = ctypes.c_float(), ctypes.c_float(), ctypes.c_int64()
    L.oracle_error_scan_reduced(0, 0x3F000000, stride, arith, 0, 1, 8, ctypes.byref(mv),
                                ctypes.byref(rv), ctypes.byref(ma), ctypes.byref(a),
                                ctypes.byref(b), ctypes.byref(n))
    return mv.value, ma.value


def failed_pins(L):
    """Names of the pins that this compiled copy of the oracle fails."""
    from oracle import exact_binary32 as ex
    bad = []
    # constants against the printed decimals
    got = np.zeros(8, np.float32)
    L.oracle_constants(0, _p(got))
    rows = {r[0]: r[2] for r in loader.coefficients() if r[1] in ("1", "both")}
    want = [np.float32(1.0 / (2.0 * float(rows["pi"])))] + [np.float32(float(rows[k])) for k in
                                                             ("ss1", "ss2", "ss3", "ss4", "cc1", "cc2", "cc3")]
    if not np.array_equal(got.view(np.uint32), np.array(want, np.float32).view(np.uint32)):
        bad.append("constants")
    # reduction invariants and ties
    rng = np.random.default_rng(1)
    x = rng.uniform(-1e4, 1e4, 4000).astype(np.float32)
    q = np.empty_like(x)
    L.oracle_reduce_f32(_p(x), _p(q), x.size)
    x1 = (x * np.float32(1.0 / (2 * math.pi))).astype(np.float32)
    if np.any(np.abs(q) > 0.5) or np.any((q + np.rint(x1)).astype(np.float32) != x1):
        bad.append("reduction")
    k = np.float32(1.0 / (2 * math.pi))
    ties = []
    for n in range(-10, 10):
        x0 = np.float32((n + 0.5) / float(k))
        for cand in (x0, np.nextafter(x0, np.float32(1e9)), np.nextafter(x0, np.float32(-1e9))):
            if np.float32(cand * k) == np.float32(n + 0.5):
                ties.append((cand, 0.5 if n % 2 == 0 else -0.5))
                break
    tq = np.empty(len(ties), np.float32)
    tx = np.array([t[0] for t in ties], np.float32)
    L.oracle_reduce_f32(_p(tx), _p(tq), tx.size)
    if not np.array_equal(tq, np.array([t[1] for t in ties], np.float32)):
        bad.append("ties")
    # accuracy and amplitude on the reduced angle (strided), both modes
    mv, ma = _scan(L, 0, 61)
    if not (mv < 4.95e-7 and ma < 1.75e-7):
        bad.append("accuracy_fused")
    mv, ma = _scan(L, 1, 61)
    if not (mv < 5.6e-7 and ma < 2.15e-7):
        bad.append("accuracy_split")
    # subnormals survive
    s, c = _sincos(L, np.array([1e-40, -1e-40], np.float32), 0)
    if np.any(s == 0):
        bad.append("subnormal")
    # exact-rational bits, both modes
    pts = np.concatenate([rng.uniform(-10, 10, 60), [1e-40, math.pi]]).astype(np.float32)
    for arith in (0, 1):
        s, c = _sincos(L, pts, arith)
        for i, v in enumerate(pts):
            if ex.pair(float(v), arith == 0, 0) != (int(s[i:i + 1].view(np.uint32)[0]),
                                                    int(c[i:i + 1].view(np.uint32)[0])):
                bad.append("exact_bits_%d" % arith)
                break
    return bad


def test_unmodified_oracle_passes_every_pin(tmp_path):
    assert failed_pins(_build(tmp_path, "clean", open(SRC).read())) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_fails_a_pin(tmp_path, name):
    src = open(SRC).read()
    old, new = MUTANTS[name]
    assert old in src, "mutation site not found: " + name
    L = _build(tmp_path, name, src.replace(old, new, 1))
    assert failed_pins(L), "no pin caught mutant " + name


# ---------------------------------------------------------------------------
# The Huygens sum's pins catch plausible mistakes in it too.

HUYGENS_MUTANTS = {
    "amp_times_r": ("float w = sq[2] / r;", "float w = sq[2] * r;"),
    "drop_dy": ("float rho2 = fmaf(dx, dx, dy2);", "float rho2 = dx * dx; (void)dy2;"),
    "path_minus_L": ("float d = rho2 / (r + j->L);", "float d = r - j->L;"),
    "path_no_L": ("float d = rho2 / (r + j->L);", "float d = rho2 / r;"),
    "phase_sign": ("float theta = fmaf(j->k, d, sq[3]);", "float theta = fmaf(j->k, d, -sq[3]);"),
    "swap_re_im": ("re = fmaf(w, cv, re);\n            im = fmaf(w, sv, im);",
                   "re = fmaf(w, sv, re);\n            im = fmaf(w, cv, im);"),
    "L2_missing": ("float r = sqrtf(rho2 + L2);", "float r = sqrtf(rho2 + j->L);"),
}


def huygens_pins_fail(L):
    import math
    from test_oracle_huygens import K, exact_field, field_bound
    fp = ctypes.POINTER(ctypes.c_float)
    L.oracle_huygens_f32.argtypes = [fp, fp, ctypes.c_int64, fp, ctypes.c_int32, ctypes.c_float,
                                     ctypes.c_float, fp, fp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    rng = np.random.default_rng(6)
    S, P = 200, 300
    src = np.stack([rng.uniform(-50, 50, S), rng.uniform(-50, 50, S), rng.uniform(0, 1, S) / S,
                    rng.uniform(-3, 3, S)], 1).astype(np.float32)
    xo = rng.uniform(-200, 200, P).astype(np.float32)
    yo = rng.uniform(-200, 200, P).astype(np.float32)
    re, im = np.empty(P, np.float32), np.empty(P, np.float32)
    L.oracle_huygens_f32(_p(xo), _p(yo), P, _p(np.ascontiguousarray(src)), S, K, 5000.0,
                         _p(re), _p(im), 0, 0, 2)
    er, ei, w, th, d = exact_field(xo, yo, src, K, 5000.0)
    return not np.all(np.hypot(re - er, im - ei) <= field_bound(w, th, d, K))


def test_unmodified_huygens_passes(tmp_path):
    assert not huygens_pins_fail(_build(tmp_path, "hclean", open(SRC).read()))


@pytest.mark.parametrize("name", sorted(HUYGENS_MUTANTS))
def test_huygens_mutant_fails_a_pin(tmp_path, name):
    src = open(SRC).read()
    old, new = HUYGENS_MUTANTS[name]
    assert old in src, "mutation site not found: " + name
    assert huygens_pins_fail(_build(tmp_path, name, src.replace(old, new, 1))), name
