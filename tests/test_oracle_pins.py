"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test targets a mistake the oracle could plausibly contain (a wrong or
mistyped coefficient, a dropped series term, a sign or factor error in the
doubling, a missing or misplaced magnitude fix, ties rounded away from zero,
flushed subnormals, contraction in the split mode) and fails on it.
"""
import math
import struct

import numpy as np
import pytest

from golden import loader

FUSED, SPLIT = 0, 1
M1, M2 = 0, 1
TWO_PI = 2.0 * math.pi


def f32_bits(v):
    return np.asarray(v, np.float32).view(np.uint32)


def ulp32(x):
    """Spacing of binary32 numbers at |x| (for x not zero)."""
    x = np.abs(np.asarray(x, np.float32))
    return (np.nextafter(x, np.float32(np.inf)) - x).astype(np.float64)


def vec_err(s, c, ang):
    ang = np.asarray(ang, np.float64)
    return np.sqrt((s.astype(np.float64) - np.sin(ang)) ** 2
                   + (c.astype(np.float64) - np.cos(ang)) ** 2)


def amp_err(s, c):
    return np.abs(1.0 - np.sqrt(s.astype(np.float64) ** 2 + c.astype(np.float64) ** 2))


# ---------------------------------------------------------------------------
# Constants: the printed decimals, rounded to binary32.


def test_constants_are_the_printed_decimals(orc):
    rows = loader.coefficients()
    order = ["ss1", "ss2", "ss3", "ss4", "cc1", "cc2", "cc3"]
    for method, tag in ((M1, "1"), (M2, "2")):
        got = orc.constants(method)
        pi_text = [r for r in rows if r[0] == "pi"][0][2]
        k = np.float32(1.0 / (2.0 * float(pi_text)))
        assert f32_bits(got[0]) == f32_bits(k)
        for j, name in enumerate(order):
            dec = [r for r in rows if r[0] == name and r[1] == tag][0][2]
            via_double = np.float32(float(dec))
            assert f32_bits(got[1 + j]) == f32_bits(via_double), (method, name)
            # decimal -> binary32 directly gives the same bits (no double rounding)
            direct = struct.unpack("<f", struct.pack("<f", float(dec)))[0]
            assert f32_bits(via_double) == f32_bits(np.float32(direct))
    # the truncated pi of the listing rounds to the same binary32 as 1/(2 pi)
    assert f32_bits(np.float32(1.0 / TWO_PI)) == f32_bits(orc.constants(M1)[0])


# ---------------------------------------------------------------------------
# Step 1: reduction modulo 1.


def test_reduction_invariants(orc):
    rng = np.random.default_rng(21)
    x = np.concatenate([rng.uniform(-10, 10, 20000), rng.uniform(-1e7, 1e7, 20000),
                        [0.0, -0.0, 1e-40, -1e-40, 3e38, -3e38]]).astype(np.float32)
    q = orc.reduce(x)
    k = orc.constants(M1)[0]
    x1 = (x * k).astype(np.float32)           # binary32 product, correctly rounded
    r = x1 - q                                 # must be the nearest integer of x1
    assert np.all(np.abs(q) <= 0.5)
    assert np.all(r == np.rint(x1))
    assert np.all((q + np.rint(x1)).astype(np.float32) == x1)
    # zero reduced angle is +0 (never -0), so the sign rules of the +0 addends
    # in the paper's form cannot change the output
    zero = q == 0
    assert np.all(np.signbit(q[zero]) == False)  # noqa: E712


def test_reduction_ties_go_to_even(orc):
    """x1 exactly half-integral: q1 = +1/2 when rint rounds down (even floor),
    -1/2 when it rounds up.  Rounding ties away from zero would give the
    opposite sign for half of them."""
    k = orc.constants(M1)[0]
    found = []
    for n in range(-40, 40):
        target = n + 0.5
        x0 = np.float32(target / float(k))
        for cand in (x0, np.nextafter(x0, np.float32(np.inf)), np.nextafter(x0, np.float32(-np.inf))):
            if np.float32(cand * k) == np.float32(target):
                found.append((cand, n))
                break
    assert len(found) > 20
    for cand, n in found:
        q = orc.reduce(np.array([cand], np.float32))[0]
        expected = 0.5 if n % 2 == 0 else -0.5   # floor n even -> rint = n
        assert q == np.float32(expected), (cand, n, q)


# ---------------------------------------------------------------------------
# Steps 2-4 on the reduced angle: accuracy against the system library.


@pytest.mark.slow
def test_exhaustive_reduced_angle_error_method1_fused(orc):
    """Every binary32 q in [0, 1/2]: matches the printed maximum vector and
    amplitude errors of the first method (the paper does not give its
    sampling; 20 % slack) and stays under a gate set just above the
    exhaustive maxima."""
    acc = loader.accuracy()
    st = orc.error_scan_reduced(0, 0x3F000000, 1, FUSED, M1, True)
    assert st["count"] == 0x3F000000 + 1
    assert abs(st["max_vec"] / acc["method1_max_vec"] - 1) < 0.2, st
    assert abs(st["max_amp"] / acc["method1_max_amp"] - 1) < 0.2, st
    assert st["max_vec"] < 4.95e-7 and st["max_amp"] < 1.75e-7, st


def test_strided_reduced_angle_error_other_modes(orc):
    acc = loader.accuracy()
    split = orc.error_scan_reduced(0, 0x3F000000, 13, SPLIT, M1, True)
    assert split["max_vec"] < 5.6e-7 and split["max_amp"] < 2.15e-7, split
    m2 = orc.error_scan_reduced(0, 0x3F000000, 13, FUSED, M2, True)
    assert abs(m2["max_vec"] / acc["method2_max_vec"] - 1) < 0.2, m2
    assert m2["max_vec"] < 4.5e-7, m2


def test_rms_over_uniform_angles_matches_paper(orc):
    """RMS vector error over angles uniform in [-pi, pi) against the double
    library at the binary32 input: 1.2e-7 (method 1) and 9.8e-8 (method 2)."""
    acc = loader.accuracy()
    v = np.random.default_rng(7).uniform(-math.pi, math.pi, 1 << 22).astype(np.float32)
    s, c = orc.sincos(v, FUSED, M1, threads=8)
    e1 = vec_err(s, c, v)
    assert abs(np.sqrt(np.mean(e1 ** 2)) / acc["method1_rms_vec"] - 1) < 0.05
    s, c = orc.sincos(v, FUSED, M2, threads=8)
    e2 = vec_err(s, c, v)
    assert abs(np.sqrt(np.mean(e2 ** 2)) / acc["method2_rms_vec"] - 1) < 0.05


def test_quarter_series_alone(orc):
    """Step 2 approximates sin and cos of pi q / 2 on [-1/2, 1/2] (a quarter of
    the reduced turn); the first method's pair is normalized to ~1e-7."""
    q = np.linspace(-0.5, 0.5, 2001).astype(np.float32)
    for method, tol_angle in ((M1, 3e-7), (M2, 5e-7)):
        es, ang = [], []
        for v in q:
            s1, c1 = orc.quarter_series(float(v), FUSED, method)
            a = math.pi * float(v) / 2
            if method == M1:
                es.append(math.hypot(s1 - math.sin(a), c1 - math.cos(a)))
            ang.append(abs(math.atan2(s1, c1) - a))
        assert max(ang) < tol_angle, (method, max(ang))
        if method == M1:
            assert max(es) < 2.5e-7
    # the second method's pair is not normalized (the paper's dagger warning)
    s1, c1 = orc.quarter_series(0.5, FUSED, M2)
    assert abs(math.hypot(s1, c1) - 1) > 1e-5


# ---------------------------------------------------------------------------
# Step 3: eq. (1) doubling, and the stability law.


def test_doubling_closed_form_and_magnitude_law(orc):
    """(a cos t, a sin t) -> (a^2 cos 2t, a^2 sin 2t): the angle error is kept
    and only the magnitude drifts (Sec. II stability analysis)."""
    rng = np.random.default_rng(3)
    for a in (1.0, 1.0 + 1e-4, 1.0 - 3e-4):
        for t in rng.uniform(-math.pi, math.pi, 200):
            s = np.float32(a * math.sin(t))
            c = np.float32(a * math.cos(t))
            s2, c2 = orc.double_angle(float(s), float(c), FUSED)
            s3, c3 = orc.double_angle(float(s2), float(c2), FUSED)
            aa = math.hypot(float(s), float(c))
            tt = math.atan2(float(s), float(c))
            assert abs(math.hypot(s2, c2) - aa ** 2) < 3e-7
            assert abs(math.remainder(math.atan2(s2, c2) - 2 * tt, TWO_PI)) < 3e-7 / aa ** 2
            assert abs(math.hypot(s3, c3) - aa ** 4) < 6e-7
            assert abs(math.remainder(math.atan2(s3, c3) - 4 * tt, TWO_PI)) < 6e-7 / aa ** 4


def test_rejected_doubling_would_mix_errors():
    """Contrast from Sec. II: with cos 2t = 1 - 2 sin^2 t the amplitude error
    leaks into the angle; the chosen form keeps it in the magnitude only.
    Checked in exact arithmetic on a drifted pair."""
    a, t = 1.0 + 1e-3, 0.7
    s, c = a * math.sin(t), a * math.cos(t)
    good = (2 * s * c, c * c - s * s)
    bad = (2 * s * c, 1 - 2 * s * s)
    assert abs(math.atan2(*good) - 2 * t) < 1e-12
    assert abs(math.atan2(*bad) - 2 * t) > 1e-4


# ---------------------------------------------------------------------------
# Step 4: the magnitude fix.


def test_magnitude_factor_closed_form(orc):
    """With |p2|^2 = 1 + e the final pair has magnitude 1 + e; the method-1
    factor 2 - |p2|^2 = 1 - e and the method-2 factor 1/(1 + e) both bring it
    back to 1 within O(e^2) (method 1) or rounding (method 2)."""
    rng = np.random.default_rng(4)
    for e in (3e-4, -2e-4, 1e-5):
        for t in rng.uniform(-math.pi, math.pi, 100):
            r = math.sqrt(1 + e)
            s2, c2 = np.float32(r * math.sin(t)), np.float32(r * math.cos(t))
            e_true = float(s2) ** 2 + float(c2) ** 2 - 1
            s3, c3 = orc.double_angle(float(s2), float(c2), FUSED)
            m1 = float(orc.magnitude_factor(float(s2), float(c2), FUSED, M1))
            m2 = float(orc.magnitude_factor(float(s2), float(c2), FUSED, M2))
            assert abs(m1 - (1 - e_true)) < 2.5e-7
            assert abs(m2 - 1 / (1 + e_true)) < 1.5e-7
            mag3 = math.hypot(s3, c3)
            assert abs(m1 * mag3 - 1) < e_true ** 2 + 4e-7
            assert abs(m2 * mag3 - 1) < 4e-7


def test_fix_removes_predicted_drift(orc):
    """Without step 4 the amplitude drifts by several 1e-7 (the paper predicts
    about 4e-7 for n = 2 doublings); with it the drift falls below 1.8e-7."""
    acc = loader.accuracy()
    unfixed = orc.error_scan_reduced(0, 0x3F000000, 29, FUSED, M1, False)
    fixed = orc.error_scan_reduced(0, 0x3F000000, 29, FUSED, M1, True)
    assert 0.5 < unfixed["max_amp"] / acc["unfixed_amp_predicted"] < 1.6, unfixed
    assert fixed["max_amp"] < 0.4 * unfixed["max_amp"]


# ---------------------------------------------------------------------------
# Symmetry, special points, special values.


def test_odd_even_symmetry_bit_exact(orc):
    rng = np.random.default_rng(5)
    q = np.concatenate([rng.uniform(0, 0.5, 50000), [0.5, 0.25, 0.125, 1e-30, 1e-42]]).astype(np.float32)
    for arith in (FUSED, SPLIT):
        for method in (M1, M2):
            sp, cp = orc.pair_from_reduced(q, arith, method)
            sn, cn = orc.pair_from_reduced(-q, arith, method)
            assert np.array_equal(f32_bits(sn), f32_bits(-sp))
            assert np.array_equal(f32_bits(cn), f32_bits(cp))


def test_special_reduced_points(orc):
    for arith in (FUSED, SPLIT):
        s, c = orc.pair_from_reduced(np.array([0.0, 0.25, -0.25, 0.125, 0.5, -0.5], np.float32), arith)
        assert s[0] == 0 and not np.signbit(s[0]) and c[0] == 1
        assert abs(s[1] - 1) <= 2 ** -23 and abs(c[1]) <= 1e-8
        assert abs(s[2] + 1) <= 2 ** -23 and abs(c[2]) <= 1e-8
        assert abs(s[3] - math.sqrt(0.5)) < 2e-7 and abs(c[3] - math.sqrt(0.5)) < 2e-7
        assert c[4] == -1 and c[5] == -1 and 0 < abs(s[4]) < 4e-7 and s[5] == -s[4]


def test_special_values(orc):
    x = np.array([np.inf, -np.inf, np.nan, 0.0, -0.0], np.float32)
    for arith in (FUSED, SPLIT):
        s, c = orc.sincos(x, arith)
        assert np.all(np.isnan(s[:3])) and np.all(np.isnan(c[:3]))
        assert np.all(s[3:] == 0) and not np.any(np.signbit(s[3:])) and np.all(c[3:] == 1)


def test_subnormals_are_kept(orc):
    """For tiny angles s = 4 fl(fl(x K) ss1) ~ x: IEEE subnormals survive
    (a flush-to-zero anywhere would give 0)."""
    x = np.array([1e-40, -1e-40, 1e-44, 2e-38, -3e-39], np.float32)
    for arith in (FUSED, SPLIT):
        s, c = orc.sincos(x, arith)
        assert np.all(c == 1)
        assert np.all(s != 0) and np.all(np.sign(s) == np.sign(x))
        assert np.all(np.abs(s.astype(np.float64) - x) <= 8 * 2.0 ** -149 + np.abs(x) * 1e-6)


def test_beyond_integer_range_reduces_to_zero(orc):
    """|x| K >= 2^23 is already an integer in binary32, so q1 = 0 and the pair
    is (0, 1): what the binary32 sequence gives, documented, not trigonometry."""
    k = float(orc.constants(M1)[0])
    x = np.array([2 ** 23 / k * 1.0001, -6e7, 1e10, -3e38], np.float32)
    for arith in (FUSED, SPLIT):
        s, c = orc.sincos(x, arith)
        assert np.all(s == 0) and np.all(c == 1)


def test_multiples_of_half_pi_within_reduction_bound(orc):
    """v = fl(k pi/2), |k| <= 64: error against the double library at v stays
    within E(v) = E_red + 2 pi |v| |K - 1/(2 pi)| + pi ulp(x1), where E_red is
    the reduced-angle maximum and the other two terms are the error of the
    binary32 constant K and the rounding of x1 = v K."""
    k32 = float(orc.constants(M1)[0])
    dk = abs(k32 - 1.0 / TWO_PI)
    v = np.array([np.float32(k * math.pi / 2) for k in range(-64, 65)], np.float32)
    x1 = (v * np.float32(k32)).astype(np.float32)
    for arith, e_red in ((FUSED, 4.95e-7), (SPLIT, 5.6e-7)):
        s, c = orc.sincos(v, arith)
        bound = e_red + TWO_PI * np.abs(v.astype(np.float64)) * dk + math.pi * np.where(x1 == 0, 0, ulp32(x1))
        err = vec_err(s, c, v)
        assert np.all(err <= bound), (err - bound).max()
        assert s[64] == 0 and c[64] == 1     # k = 0


@pytest.mark.parametrize("span", [8 * math.pi, 100 * math.pi, 1e4])
def test_large_angle_error_within_bound(orc, span):
    k32 = float(orc.constants(M1)[0])
    dk = abs(k32 - 1.0 / TWO_PI)
    v = np.random.default_rng(int(span)).uniform(-span, span, 200000).astype(np.float32)
    x1 = (v * np.float32(k32)).astype(np.float32)
    s, c = orc.sincos(v, FUSED)
    bound = 4.95e-7 + TWO_PI * np.abs(v.astype(np.float64)) * dk + math.pi * np.where(x1 == 0, 0, ulp32(x1))
    assert np.all(vec_err(s, c, v) <= bound)


def test_seam_only_at_the_wrap(orc):
    """The error (s, c) - (sin, cos) averaged over blocks of 1024 consecutive
    angles on a dense grid of [-4, 4] has no jump anywhere (in particular not
    at the multiples of pi/4, where quadrant-based reductions switch
    formulas), except at the wrap v = +-pi (Sec. II smoothness remark).
    Elsewhere a jump can only come from the rounded magnitude factor moving by
    one unit near 1, bounded by 2^-23."""
    v = np.linspace(-4, 4, 1 << 23).astype(np.float32)
    s, c = orc.sincos(v, FUSED, threads=8)
    vd = v.astype(np.float64)
    es, ec = s - np.sin(vd), c - np.cos(vd)
    B = 1024
    bs = es.reshape(-1, B).mean(1)
    bc = ec.reshape(-1, B).mean(1)
    centers = vd.reshape(-1, B).mean(1)
    jump = np.hypot(np.diff(bs), np.diff(bc))
    mid = 0.5 * (centers[1:] + centers[:-1])
    near_wrap = np.abs(np.abs(mid) - math.pi) < 2e-3
    assert jump[near_wrap].max() > 2.5e-7
    assert jump[~near_wrap].max() <= 2.0 ** -23
    for k in range(-5, 6):
        if abs(k) == 4:
            continue
        near = np.abs(mid - k * math.pi / 4) < 5e-3
        assert jump[near].max() < 3e-8, k


# ---------------------------------------------------------------------------
# The compiled oracle's bits against an exact-rational re-evaluation.


def _probe_points():
    rng = np.random.default_rng(9)
    k32 = 1.0 / (2.0 * 3.1415926536)
    ties = [np.float32((n + 0.5) / k32) for n in range(-6, 6)]
    pts = np.concatenate([
        rng.uniform(-10, 10, 600), rng.uniform(-1e4, 1e4, 300), rng.uniform(-1e-3, 1e-3, 100),
        ties, [0.0, -0.0, 1e-40, -1e-40, 1e-45, 2e-38, math.pi, -math.pi, math.pi / 2,
               math.pi / 4, 6e7, -6e7, 3e38],
        np.float32(math.pi) + np.arange(-20, 20) * np.float32(2 ** -22),
    ]).astype(np.float32)
    return pts


@pytest.mark.parametrize("arith", [FUSED, SPLIT])
@pytest.mark.parametrize("method", [M1, M2])
def test_compiled_oracle_matches_exact_rational(orc, arith, method):
    from oracle import exact_binary32 as ex
    x = _probe_points()
    s, c = orc.sincos(x, arith, method)
    sb, cb = f32_bits(s), f32_bits(c)
    for i, v in enumerate(x):
        assert ex.pair(float(v), arith == FUSED, method) == (int(sb[i]), int(cb[i])), float(v)


@pytest.mark.parametrize("method", [M1, M2])
def test_altivec_form_gives_the_same_bits(orc, method):
    """The +0 addends and the negated multiply-subtract of the AltiVec form
    change no output bit (fused arithmetic)."""
    from oracle import exact_binary32 as ex
    x = _probe_points()[::3]
    s, c = orc.sincos(x, FUSED, method)
    sb, cb = f32_bits(s), f32_bits(c)
    for i, v in enumerate(x):
        assert ex.pair_altivec_form(float(v), method) == (int(sb[i]), int(cb[i])), float(v)


def test_exact_rounding_helper_against_hardware():
    """The exact rounding rule reproduces numpy's binary32 products and sums
    (so the re-evaluation above is itself pinned)."""
    from fractions import Fraction
    from oracle import exact_binary32 as ex
    rng = np.random.default_rng(12)
    a = rng.standard_normal(3000).astype(np.float32) * np.float32(2.0) ** rng.integers(-140, 60, 3000).astype(np.float32)
    b = rng.standard_normal(3000).astype(np.float32)
    for x, y in zip(a, b):
        pa, pb = ex.F32.from_float(float(x)), ex.F32.from_float(float(y))
        assert ex.mul(pa, pb).bits() == int(f32_bits(np.float32(x * y)))
        assert ex.add(pa, pb).bits() == int(f32_bits(np.float32(x + y)))
    assert ex.round_binary32(Fraction(1, 2 ** 150), False).bits() == 0          # tie to even -> 0
    assert ex.round_binary32(Fraction(3, 2 ** 151), False).bits() == 1          # above the tie -> min subnormal
