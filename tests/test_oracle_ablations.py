"""The stability argument of Sec. II, shown numerically with the oracle's
ablations: with the doubling of eq. (1) the angle error of the series is
carried through unchanged and only the magnitude drifts, so the magnitude
fix (in the listing's form or the text's) leaves the angle alone; with the
rejected eq. (2) the amplitude error leaks into the angle."""
import math

import numpy as np
import pytest

import oracle

Q = np.linspace(0.0, 0.5, 20001).astype(np.float32)


def _errors(variant, arith=oracle.FUSED):
    ang, amp = [], []
    for q in Q:
        s, c = oracle.pair_variant(float(q), arith, oracle.METHOD1, variant)
        a = math.atan2(float(s), float(c))
        ang.append(abs(math.remainder(a - 2 * math.pi * float(q), 2 * math.pi)))
        amp.append(abs(1.0 - math.hypot(float(s), float(c))))
    return np.array(ang), np.array(amp)


@pytest.fixture(scope="module")
def errs(orc):
    return {v: _errors(v) for v in (oracle.VARIANT_LISTING, oracle.VARIANT_NO_FIX,
                                    oracle.VARIANT_TEXT_FIX, oracle.VARIANT_EQ2)}


def test_listing_variant_is_the_method(orc):
    for q in Q[::97]:
        assert oracle.pair_variant(float(q)) == tuple(
            v[0] for v in oracle.pair_from_reduced(np.array([q], np.float32)))


def test_fix_changes_magnitude_not_angle(errs):
    """eq. (1): the angle error is the same with and without the fix (to a
    rounding of the final scaling), only the amplitude error differs."""
    ang_fix, amp_fix = errs[oracle.VARIANT_LISTING]
    ang_none, amp_none = errs[oracle.VARIANT_NO_FIX]
    assert abs(ang_fix.max() - ang_none.max()) < 2e-8
    assert np.sqrt(np.mean((ang_fix - ang_none) ** 2)) < 3e-8
    assert amp_none.max() > 3 * amp_fix.max()


def test_text_form_fix_agrees_to_first_order(errs):
    """(3 - s^2 - c^2)/2 on the final pair and 2 - |p2|^2 after the first
    doubling agree to first order: same angles, both remove the drift."""
    ang_l, amp_l = errs[oracle.VARIANT_LISTING]
    ang_t, amp_t = errs[oracle.VARIANT_TEXT_FIX]
    assert abs(ang_l.max() - ang_t.max()) < 2e-8
    assert amp_t.max() < 1.8e-7 and amp_l.max() < 1.8e-7


def test_rejected_doubling_mixes_amplitude_into_angle(errs):
    """eq. (2) (cos 2a = 1 - 2 sin^2 a): the angle error grows; the magnitude
    fix cannot repair it."""
    ang_1, _ = errs[oracle.VARIANT_LISTING]
    ang_2, amp_2 = errs[oracle.VARIANT_EQ2]
    assert ang_2.max() > 1.4 * ang_1.max()
    assert np.sqrt(np.mean(ang_2 ** 2)) > 1.6 * np.sqrt(np.mean(ang_1 ** 2))
    assert amp_2.max() > 2 * errs[oracle.VARIANT_LISTING][1].max()


def test_variant_scans(orc):
    """The whole reduced range (strided): the listing's and the text's fix
    give the same maximum vector error; eq. (2) is clearly worse."""
    st = {v: orc.error_scan_variant(0, 0x3F000000, 31, oracle.FUSED, oracle.METHOD1, v)
          for v in (oracle.VARIANT_LISTING, oracle.VARIANT_TEXT_FIX, oracle.VARIANT_EQ2)}
    assert abs(st[oracle.VARIANT_TEXT_FIX]["max_vec"] / st[oracle.VARIANT_LISTING]["max_vec"] - 1) < 0.02
    assert st[oracle.VARIANT_EQ2]["max_vec"] > 1.4 * st[oracle.VARIANT_LISTING]["max_vec"]
