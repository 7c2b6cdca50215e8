"""Pins of the oracle's ablation paths (the rejected eq. (2) doubling, the
text's magnitude factor, the general form with n = 0 doublings), written as
functions of a loaded oracle library so that the mutant tests can run them
against deliberately broken copies.

Each pin compares the compiled oracle with something other than itself:
- the closed forms of the stability analysis of Sec. II, evaluated in double
  precision through a different route (trigonometry of the pair's own
  magnitude and angle, not the doubling formula);
- the exact-rational re-evaluation (``oracle.exact_binary32``), which
  composes the steps on its own, with IEEE rounding written out.

Every function returns the list of pin names that the library fails.
"""
import ctypes
import math

import numpy as np

FUSED, SPLIT = 0, 1
VARIANT_NO_FIX, VARIANT_TEXT_FIX, VARIANT_EQ2 = 1, 2, 3
ULP1 = 2.0 ** -23          # spacing of binary32 just above 1


def _bind(L):
    fp = ctypes.POINTER(ctypes.c_float)
    c_int = ctypes.c_int
    L.oracle_double_angle_eq2.argtypes = [ctypes.c_float, ctypes.c_float, c_int, fp, fp]
    L.oracle_quarter_series.argtypes = [ctypes.c_float, c_int, c_int, fp, fp]
    L.oracle_pair_variant.argtypes = [ctypes.c_float, c_int, c_int, c_int, fp, fp]
    L.oracle_pair_general.argtypes = [ctypes.c_float, c_int, c_int, fp, c_int, fp, c_int, c_int,
                                      fp, fp]
    return L


def _two(fn, *args):
    a, b = ctypes.c_float(), ctypes.c_float()
    fn(*args, ctypes.byref(a), ctypes.byref(b))
    return np.float32(a.value), np.float32(b.value)


def _bits(v):
    return int(np.float32(v).view(np.uint32))


def eq2_double(L, s, c, arith):
    return _two(L.oracle_double_angle_eq2, ctypes.c_float(s), ctypes.c_float(c), arith)


def variant(L, x, arith, method, which):
    return _two(L.oracle_pair_variant, ctypes.c_float(x), arith, method, which)


def general(L, x, ndoub, ss, cc, arith, fix):
    ss = np.ascontiguousarray(ss, np.float32)
    cc = np.ascontiguousarray(cc, np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    return _two(L.oracle_pair_general, ctypes.c_float(x), arith, ndoub, ss.ctypes.data_as(fp),
                ss.size, cc.ctypes.data_as(fp), cc.size, int(fix))


# Planted magnitudes: far from 1, where eq. (2) and eq. (1) differ widely,
# and near 1, where the method works.
DRIFTS = (0.5, 0.9, 0.999, 1 - 1e-5, 1.0, 1 + 1e-5, 1.001, 1.1, 2.0)


def eq2_closed_form(L):
    """Sec. II: a pair (a sin t, a cos t) doubled with eq. (2) becomes
    (a^2 sin 2t, a^2 cos 2t + (1 - a^2)).  The right-hand side is evaluated
    in double from the binary32 pair's own a^2 = s^2 + c^2 and t = atan2(s, c).
    Rounding bound: the cosine is one or two binary32 roundings of values of
    size at most 1 + 2a^2, the sine one rounding of 2sc (doubling is exact)."""
    _bind(L)
    t = np.linspace(-math.pi, math.pi, 721)
    bad = []
    for arith in (FUSED, SPLIT):
        worst = 0.0
        for a in DRIFTS:
            s32 = (a * np.sin(t)).astype(np.float32)
            c32 = (a * np.cos(t)).astype(np.float32)
            a2 = s32.astype(np.float64) ** 2 + c32.astype(np.float64) ** 2
            th = np.arctan2(s32.astype(np.float64), c32.astype(np.float64))
            want_s = a2 * np.sin(2 * th)
            want_c = a2 * np.cos(2 * th) + (1 - a2)
            tol_c = 2 * ULP1 * (1 + 2 * a2) + 1e-14
            tol_s = 2 * ULP1 * a2 + 1e-14
            for i in range(t.size):
                gs, gc = eq2_double(L, float(s32[i]), float(c32[i]), arith)
                es = abs(float(gs) - want_s[i]) / tol_s[i]
                ec = abs(float(gc) - want_c[i]) / tol_c[i]
                worst = max(worst, es, ec)
        if not worst <= 1.0:
            bad.append("eq2_closed_form_%d" % arith)
    return bad


def _series_pair(L, x, method, arith):
    return _two(L.oracle_quarter_series, ctypes.c_float(x), arith, method)


def eq2_model(L, arith=FUSED, method=0, npts=4001):
    """The eq. (2) variant against the closed form of Sec. II applied twice
    in double to the binary32 series pair (angle pi x / 2 + d, magnitude
    a = 1 + e): the model gives the angle that eq. (2) itself produces (the
    magnitude factor cannot turn the pair) and, with the method's factor
    read from the model's pair after the first doubling (2 - |p|^2 or
    1 / |p|^2), the final magnitude.
    Angle: the variant stays within the rounding of two binary32 doublings of
    the model: each rounds (s, c) by at most (1 + 2a^2) 2^-24 ~ 3.6e-7 in the
    cosine and 1.2e-7 in the sine, the second doubles the first one's error,
    and the final scaling adds 2 * 2^-24: (2 + 1) * 3.8e-7 + 1.2e-7 < 1.3e-6.
    This bounds the variant's angle error from above by the model's plus
    1.3e-6.  Magnitude: within the same budget plus the factor's roundings
    (relative 2e-6 in all).  Returns (failures, max model angle error, max
    variant angle error)."""
    _bind(L)
    xs = np.linspace(-0.5, 0.5, npts).astype(np.float32)
    worst_dev = worst_mag = 0.0
    err_model = err_oracle = 0.0
    for x in xs:
        qs, qc = _series_pair(L, float(x), method, arith)
        s, c = float(qs), float(qc)
        mags = []
        for _ in range(2):
            a2 = s * s + c * c
            th = math.atan2(s, c)
            s, c = a2 * math.sin(2 * th), a2 * math.cos(2 * th) + (1 - a2)
            mags.append(s * s + c * c)
        factor = 2.0 - mags[0] if method == 0 else 1.0 / mags[0]
        model = math.atan2(s, c)
        model_mag = math.sqrt(mags[1]) * factor
        gs, gc = variant(L, float(x), arith, method, VARIANT_EQ2)
        got = math.atan2(float(gs), float(gc))
        ref = 2 * math.pi * float(x)
        worst_dev = max(worst_dev, abs(math.remainder(got - model, 2 * math.pi)))
        worst_mag = max(worst_mag, abs(math.hypot(float(gs), float(gc)) / model_mag - 1))
        err_model = max(err_model, abs(math.remainder(model - ref, 2 * math.pi)))
        err_oracle = max(err_oracle, abs(math.remainder(got - ref, 2 * math.pi)))
    bad = []
    if not (worst_dev <= 1.3e-6 and err_oracle <= err_model + 1.3e-6):
        bad.append("eq2_angle_%d_%d" % (arith, method))
    if not worst_mag <= 2e-6:
        bad.append("eq2_magnitude_%d_%d" % (arith, method))
    return bad, err_model, err_oracle


def text_factor_closed_form(L):
    """The text's factor (Sec. II): the final pair p with |p|^2 = 1 + alpha is
    multiplied by 1 - alpha/2 = (3 - |p|^2)/2.  Checked against that product
    in double from the unfixed binary32 pair, within the roundings of the
    factor (three operations on values below 3) and of the two products, and
    the fixed magnitude within 1.8e-7 of 1 (the printed amplitude error)."""
    _bind(L)
    bad = []
    xs = np.linspace(-0.5, 0.5, 1201).astype(np.float32)
    for arith in (FUSED, SPLIT):
        for method in (0, 1):
            for x in xs:
                us, uc = variant(L, float(x), arith, method, VARIANT_NO_FIX)
                fs, fc = variant(L, float(x), arith, method, VARIANT_TEXT_FIX)
                m = (3.0 - float(us) ** 2 - float(uc) ** 2) / 2
                tol = 6 * 2.0 ** -24
                if (abs(float(fs) - m * float(us)) > tol or abs(float(fc) - m * float(uc)) > tol
                        or (method == 0 and abs(math.hypot(float(fs), float(fc)) - 1) > 1.8e-7)):
                    bad.append("text_factor_%d_%d" % (arith, method))
                    break
    return bad


def general_n0(L, ss, cc):
    """No doubling (n = 0): the series pair p itself is fixed with the text's
    (3 - |p|^2)/2.  Checked three ways: the product in double from the
    unfixed binary32 pair within the roundings (as for the text's factor);
    the fixed magnitude within 2e-7 of 1 (one Newton step leaves O(e^2) of a
    series drift e below 4e-7, plus roundings of the factor and products);
    the angle unchanged from the unfixed pair's within 2 * 2^-24 (a common
    factor cannot turn the pair; each product rounds once)."""
    _bind(L)
    bad = []
    xs = np.linspace(-0.5, 0.5, 2001).astype(np.float32)
    for arith in (FUSED, SPLIT):
        for x in xs:
            us, uc = general(L, float(x), 0, ss, cc, arith, False)
            fs, fc = general(L, float(x), 0, ss, cc, arith, True)
            m = (3.0 - float(us) ** 2 - float(uc) ** 2) / 2
            tol = 6 * 2.0 ** -24
            if abs(float(fs) - m * float(us)) > tol or abs(float(fc) - m * float(uc)) > tol:
                bad.append("n0_closed_form_%d" % arith)
                break
            if abs(math.hypot(float(fs), float(fc)) - 1) > 2e-7:
                bad.append("n0_magnitude_%d" % arith)
                break
            turn = math.remainder(math.atan2(float(fs), float(fc)) -
                                  math.atan2(float(us), float(uc)), 2 * math.pi)
            if abs(turn) > 2 * 2.0 ** -24 * 1.5:
                bad.append("n0_angle_%d" % arith)
                break
    return bad


def exact_ablation_bits(L, ss_by_n):
    """Bit equality with the exact-rational composition of the same steps
    (oracle.exact_binary32): the eq. (2), no-fix and text-fix variants in both
    arithmetics and methods, and the general form for the given doubling
    counts with and without the fix."""
    from oracle import exact_binary32 as ex
    _bind(L)
    bad = []
    rng = np.random.default_rng(11)
    xs = np.concatenate([rng.uniform(-0.5, 0.5, 40), [0.0, 0.25, -0.25, 0.5, -0.5, 1e-40,
                                                       0.125]]).astype(np.float32)
    for arith in (FUSED, SPLIT):
        fused = arith == FUSED
        for method in (0, 1):
            for which, v in (("no_fix", VARIANT_NO_FIX), ("text_fix", VARIANT_TEXT_FIX),
                             ("eq2", VARIANT_EQ2)):
                for x in xs:
                    got = variant(L, float(x), arith, method, v)
                    if ex.variant(float(x), fused, method, which) != tuple(map(_bits, got)):
                        bad.append("exact_%s_%d_%d" % (which, arith, method))
                        break
        for n, (ss, cc) in ss_by_n.items():
            for fix in (True, False):
                for x in xs:
                    got = general(L, float(x), n, ss, cc, arith, fix)
                    if ex.pair_general(float(x), n, ss, cc, fused, fix) != tuple(map(_bits, got)):
                        bad.append("exact_general_%d_%d_%d" % (n, int(fix), arith))
                        break
    return bad


def general_fix_holds(L, ss_by_n):
    """With the fix read before the last doubling, the magnitude stays within
    1.8e-7 of 1 (the printed amplitude error) at every doubling count."""
    _bind(L)
    bad = []
    xs = np.linspace(0.0, 0.5, 3001).astype(np.float32)
    for n, (ss, cc) in ss_by_n.items():
        worst = 0.0
        for x in xs:
            fs, fc = general(L, float(x), n, ss, cc, FUSED, True)
            worst = max(worst, abs(math.hypot(float(fs), float(fc)) - 1))
        if worst > 1.8e-7:
            bad.append("general_fix_%d" % n)
    return bad
