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
    "drop_ss4": ("const float sin_coef[4] = {k.ss1, k.ss2, k.ss3, k.ss4};",
                 "const float sin_coef[4] = {k.ss1, k.ss2, k.ss3, 0.0f};"),
    "drop_cc3": ("const float cos_coef[4] = {1.0f, k.cc1, k.cc2, k.cc3};",
                 "const float cos_coef[4] = {1.0f, k.cc1, k.cc2, 0.0f};"),
    "cc1_cc2_swapped": ("const float cos_coef[4] = {1.0f, k.cc1, k.cc2, k.cc3};",
                        "const float cos_coef[4] = {1.0f, k.cc2, k.cc1, k.cc3};"),
    "ss3_digit_typo": ("k.ss3 = (float)0.0796819754;", "k.ss3 = (float)0.0769819754;"),
    "horner_order": ("for (int k = n - 2; k >= 0; k--)\n        p = mul_add(x2, p, coef[k], arith);",
                     "for (int k = 0; k <= n - 2; k++)\n        p = mul_add(x2, p, coef[k], arith);"),
    "doubling_plus": ("*c_out = mul_sub_from(s, s, cos_sq, arith);",
                      "*c_out = mul_add(s, s, cos_sq, arith);"),
    "doubling_no_two": ("*c_out = mul_sub_from(s, s, cos_sq, arith);\n    float sin_cos = s * c;\n"
                        "    *s_out = 2.0f * sin_cos;",
                        "*c_out = mul_sub_from(s, s, cos_sq, arith);\n    float sin_cos = s * c;\n"
                        "    *s_out = sin_cos;"),
    "rejected_doubling": ("*c_out = mul_sub_from(s, s, cos_sq, arith);",
                          "(void)cos_sq; *c_out = mul_sub_from(2.0f * s, s, 1.0f, arith);"),
    "one_doubling": ("oracle_double_angle(hs, hc, arith, &fs, &fc);      /* angle 2 pi x   */",
                     "fs = hs; fc = hc;"),
    "no_fix": ("/* angle 2 pi x   */\n    *s = fs * m;\n    *c = fc * m;",
               "/* angle 2 pi x   */\n    (void)m;\n    *s = fs;\n    *c = fc;"),
    "fix_sign": ("return mul_sub_from(s, s, two_less_cos_sq, arith);",
                 "return mul_add(s, s, two_less_cos_sq, arith);"),
    "ties_away": ("float whole = rintf(turns);", "float whole = roundf(turns);"),
    "truncate": ("float whole = rintf(turns);", "float whole = truncf(turns);"),
    "reduce_sign": ("return turns - whole;", "return whole - turns;"),
    "pi_digits": ("(float)(1.0 / (2.0 * 3.1415926536))", "(float)(1.0 / (2.0 * 3.14159))"),
    "split_fuses": ("float p = a * b;\n    return p + c;", "return fmaf(a, b, c);"),
    "fused_splits": ("return fmaf(a, b, c);\n    float p = a * b;\n    return p + c;",
                     "{ float p = a * b; return p + c; }"),
    "flush_subnormal": ("float turns = theta * reduction_constant();",
                        "float turns = theta * reduction_constant();\n"
                        "    if (fabsf(turns) < 1.17549435e-38f) turns = 0.0f;"),
    "fix_before_doubling": ("/* angle 2 pi x   */\n    *s = fs * m;\n    *c = fc * m;",
                            "/* angle 2 pi x   */\n"
                            "    oracle_double_angle(hs * m, hc * m, arith, s, c);"),
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
    assert src.count(old) == 1, "mutation site not found or not unique: " + name
    L = _build(tmp_path, name, src.replace(old, new, 1))
    assert failed_pins(L), "no pin caught mutant " + name


# ---------------------------------------------------------------------------
# The Huygens sum's pins catch plausible mistakes in it too.

I12 = " " * 12  # the indentation of the term's branches: sites in code, not in comments
HUYGENS_MUTANTS = {
    "amp_times_r": (I12 + "w = sq[2] * (e * g);", I12 + "w = sq[2] * r;"),
    "weight_drops_e": (I12 + "w = sq[2] * (e * g);", I12 + "w = sq[2] * g;"),
    "path_drops_r": (I12 + "d = rho2 * (r * g);", I12 + "d = rho2 * g;"),
    "path_overflowing_order": (I12 + "d = rho2 * (r * g);", I12 + "d = (rho2 * r) * g;"),
    "recip_drops_r": ("float x = r * e;", "float x = e;"),
    "recip_of_r_only": ("float x = r * e;", "float x = r * r;"),
    "fallback_path_no_L": ("} else {\n" + I12 + "d = rho2 / e;",
                           "} else {\n" + I12 + "d = rho2 / r;"),
    "fallback_amp_times_r": (I12 + "w = sq[2] / r;", I12 + "w = sq[2] * r;"),
    "drop_dy": ("float rho2 = fmaf(dx, dx, dy2);", "float rho2 = dx * dx; (void)dy2;"),
    "path_minus_L": (I12 + "d = rho2 * (r * g);", I12 + "d = r - j->L;"),
    "path_no_L": ("float e = r + j->L;", "float e = r;"),
    "phase_sign": ("float theta = fmaf(j->k, d, sq[3]);", "float theta = fmaf(j->k, d, -sq[3]);"),
    "swap_re_im": ("re = fmaf(w, cv, re);\n        im = fmaf(w, sv, im);",
                   "re = fmaf(w, sv, re);\n        im = fmaf(w, cv, im);"),
    "L2_missing": ("float r = sqrtf(rho2 + L2);", "float r = sqrtf(rho2 + j->L);"),
    "one_block": ("#define HUYGENS_BLOCKS 4", "#define HUYGENS_BLOCKS 1"),
    "block_size_floor": ("const int32_t per = (int32_t)(((int64_t)j->S + j->blocks - 1) / j->blocks);",
                         "const int32_t per = (int32_t)((int64_t)j->S / j->blocks);"),
    "block_start_skips": ("huygens_block_sum(j, i, first, last, &bre, &bim);",
                          "huygens_block_sum(j, i, first + (b > 0), last, &bre, &bim);"),
    "last_block_only": ("            if (b == 0) {\n                re = bre;",
                        "            if (1) {\n                re = bre;"),
}


def huygens_pins_fail(L):
    import math
    from test_oracle_huygens import EXTREME_CASES, K, exact_field, extreme_case, field_bound
    fp = ctypes.POINTER(ctypes.c_float)
    L.oracle_huygens_f32.argtypes = [fp, fp, ctypes.c_int64, fp, ctypes.c_int32, ctypes.c_float,
                                     ctypes.c_float, fp, fp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.oracle_huygens_blocks_f32.argtypes = [fp, fp, ctypes.c_int64, fp, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_float, ctypes.c_float, fp,
                                            fp, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    rng = np.random.default_rng(6)
    S, P = 203, 300
    src = np.stack([rng.uniform(-50, 50, S), rng.uniform(-50, 50, S), rng.uniform(0, 1, S) / S,
                    rng.uniform(-3, 3, S)], 1).astype(np.float32)
    xo = rng.uniform(-200, 200, P).astype(np.float32)
    yo = rng.uniform(-200, 200, P).astype(np.float32)

    def blocked(tab, blocks):
        tab = np.ascontiguousarray(tab, np.float32)
        re, im = np.empty(P, np.float32), np.empty(P, np.float32)
        L.oracle_huygens_blocks_f32(_p(xo), _p(yo), P, _p(tab) if tab.size else None,
                                    tab.shape[0], blocks, K, 5000.0, _p(re), _p(im), 0, 0, 2)
        return re, im
    re, im = np.empty(P, np.float32), np.empty(P, np.float32)
    L.oracle_huygens_f32(_p(xo), _p(yo), P, _p(np.ascontiguousarray(src)), S, K, 5000.0,
                         _p(re), _p(im), 0, 0, 2)
    er, ei, w, th, d = exact_field(xo, yo, src, K, 5000.0)
    if not np.all(np.hypot(re - er, im - ei) <= field_bound(w, th, d, K)):
        return True
    # the ends of the range: one reciprocal with r near 2^50, two divisions
    # where r (r + L) leaves the normal range
    for name in sorted(EXTREME_CASES):
        exo, eyo, esrc, ek, eL = extreme_case(name)
        ere, eim = np.empty(exo.size, np.float32), np.empty(exo.size, np.float32)
        L.oracle_huygens_f32(_p(exo), _p(eyo), exo.size, _p(np.ascontiguousarray(esrc)),
                             esrc.shape[0], ek, eL, _p(ere), _p(eim), 0, 0, 2)
        er, ei, w, th, d = exact_field(exo, eyo, esrc, ek, eL)
        err = np.hypot(ere.astype(np.float64) - er, eim.astype(np.float64) - ei)
        if not np.all(err <= field_bound(w, th, d, ek)):
            return True
    # the structure: four blocks of ceil(S/4), plain sums, added in block order
    per = -(-S // 4)
    wr = wi = None
    for b in range(4):
        br, bi = blocked(src[min(S, b * per):min(S, (b + 1) * per)], 1)
        wr, wi = (br, bi) if wr is None else ((wr + br).astype(np.float32),
                                             (wi + bi).astype(np.float32))
    return not (np.array_equal(re.view(np.uint32), wr.view(np.uint32)) and
                np.array_equal(im.view(np.uint32), wi.view(np.uint32)))


def test_unmodified_huygens_passes(tmp_path):
    assert not huygens_pins_fail(_build(tmp_path, "hclean", open(SRC).read()))


@pytest.mark.parametrize("name", sorted(HUYGENS_MUTANTS))
def test_huygens_mutant_fails_a_pin(tmp_path, name):
    src = open(SRC).read()
    old, new = HUYGENS_MUTANTS[name]
    assert src.count(old) == 1, "mutation site not found or not unique: " + name
    assert huygens_pins_fail(_build(tmp_path, name, src.replace(old, new, 1))), name


# ---------------------------------------------------------------------------
# The ablation paths of Sec. II: the rejected eq. (2) doubling, the text's
# magnitude factor and the general form with n = 0 doublings.

ABLATION_MUTANTS = {
    "eq2_cos_for_sin": ("float twice_sin = 2.0f * s;\n    *c_out = mul_sub_from(twice_sin, s, 1.0f, arith);",
                        "float twice_sin = 2.0f * c;\n    *c_out = mul_sub_from(twice_sin, c, 1.0f, arith);"),
    "eq2_sign": ("*c_out = mul_sub_from(twice_sin, s, 1.0f, arith);",
                 "*c_out = mul_add(twice_sin, s, 1.0f, arith);"),
    "eq2_no_two": ("float twice_sin = 2.0f * s;", "float twice_sin = s;"),
    "eq2_sine_no_two": ("*s_out = 2.0f * sin_cos;\n}\n\n/* Magnitude factor",
                        "*s_out = sin_cos;\n}\n\n/* Magnitude factor"),
    "eq2_second_doubling_eq1": ("oracle_double_angle_eq2(hs, hc, arith, &fs, &fc);",
                                "oracle_double_angle(hs, hc, arith, &fs, &fc);"),
    "eq2_factor_from_series": ("float m = oracle_magnitude_factor(hs, hc, arith, method);\n"
                               "        oracle_double_angle_eq2",
                               "float m = oracle_magnitude_factor(qs, qc, arith, method);\n"
                               "        oracle_double_angle_eq2"),
    "text_factor_unhalved": ("return 0.5f * h;", "return h;"),
    "text_factor_two": ("float three_less_cos_sq = mul_sub_from(c, c, 3.0f, arith);",
                        "float three_less_cos_sq = mul_sub_from(c, c, 2.0f, arith);"),
    "text_factor_sign": ("float h = mul_sub_from(s, s, three_less_cos_sq, arith);",
                         "float h = mul_add(s, s, three_less_cos_sq, arith);"),
    "n0_no_fix": ("if (ndoub == 0 && fix)\n        m = text_factor(ps, pc, arith);",
                  "if (ndoub == 0 && fix)\n        m = 1.0f;"),
    "n0_listing_factor": ("if (ndoub == 0 && fix)\n        m = text_factor(ps, pc, arith);",
                          "if (ndoub == 0 && fix)\n"
                          "        m = oracle_magnitude_factor(ps, pc, arith, ORACLE_METHOD1);"),
    "general_fix_from_series": ("if (fix && d == ndoub - 1)", "if (fix && d == 0)"),
    "general_cos_no_one": ("float pc = mul_add(x2, horner(x2, cc, nc, arith), 1.0f, arith);",
                           "float pc = x2 * horner(x2, cc, nc, arith);"),
}


@pytest.fixture(scope="module")
def ablation_series():
    from oracle import series_fit
    return {n: series_fit.fit_series(n, ns, nc) for n, ns, nc in ((0, 6, 6), (1, 5, 4), (3, 3, 3),
                                                                  (4, 3, 2))}


def ablation_pins_fail(L, series):
    import ablation_pins as ap
    bad = ap.eq2_closed_form(L)
    for arith in (0, 1):
        for method in (0, 1):
            bad += ap.eq2_model(L, arith, method, npts=1001)[0]
    bad += ap.text_factor_closed_form(L)
    bad += ap.general_n0(L, *series[0])
    bad += ap.exact_ablation_bits(L, {n: series[n] for n in (0, 1, 3)})
    bad += ap.general_fix_holds(L, {n: series[n] for n in (1, 3, 4)})
    return bad


def test_unmodified_oracle_passes_ablation_pins(tmp_path, ablation_series):
    assert ablation_pins_fail(_build(tmp_path, "aclean", open(SRC).read()), ablation_series) == []


@pytest.mark.parametrize("name", sorted(ABLATION_MUTANTS))
def test_ablation_mutant_fails_a_pin(tmp_path, name, ablation_series):
    src = open(SRC).read()
    old, new = ABLATION_MUTANTS[name]
    assert src.count(old) == 1, "mutation site not unique: " + name
    bad = ablation_pins_fail(_build(tmp_path, name, src.replace(old, new)), ablation_series)
    assert bad, "no pin caught mutant " + name
