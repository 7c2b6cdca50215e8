"""Exact-rational re-evaluation of the sine-cosine pair, for checking the
compiled oracle's bits.

TEST INFRASTRUCTURE (see the package docstring).

Every binary32 value is held as a Python ``Fraction`` (plus an explicit sign
for zeros), every operation is carried out exactly, and the result is rounded
to binary32 by the IEEE 754 rule written out below: round to nearest, ties to
even, with gradual underflow (subnormals) and overflow to infinity.  Nothing
here calls a floating-point unit for the arithmetic of the method, so a
contraction, an excess-precision register or a flush-to-zero in the compiled
oracle shows up as a bit difference.

Besides the reading of the compiled oracle (a product is a plain product, the
negative multiply-subtract is fusedMultiplyAdd(-a, b, c)), the function
``pair_altivec_form`` evaluates the multiply-adds the way the AltiVec form of
the paper's Fig. 1 writes them: every plain product as a fused multiply-add
with a +0 addend, and the negative multiply-subtract as the negation of
(a*b - c).  Equal bits from the two show that the readings change no output.
Finite inputs only.
"""
from __future__ import annotations

import struct
from fractions import Fraction

_EMIN = -126           # smallest normal exponent of binary32
_P = 24                # precision in bits
_MAXF = (2 - Fraction(1, 2 ** 23)) * Fraction(2) ** 127


class F32:
    """A binary32 value: exact rational magnitude with a sign (for zeros)."""

    __slots__ = ("v", "neg", "inf")

    def __init__(self, v: Fraction, neg: bool | None = None, inf: bool = False):
        self.v = Fraction(v)
        self.neg = (self.v < 0) if neg is None else neg
        self.inf = inf

    @staticmethod
    def from_float(x: float) -> "F32":
        x = float(struct.unpack("<f", struct.pack("<f", x))[0])
        if x != x or x in (float("inf"), float("-inf")):
            raise ValueError("finite values only")
        neg = struct.pack("<f", x)[3] & 0x80 != 0
        return F32(Fraction(x), neg)

    def to_float(self) -> float:
        if self.inf:
            return float("-inf") if self.neg else float("inf")
        if self.v == 0:
            return -0.0 if self.neg else 0.0
        return float(self.v)  # exact: every binary32 is a binary64

    def bits(self) -> int:
        return struct.unpack("<I", struct.pack("<f", self.to_float()))[0]


def round_binary32(v: Fraction, zero_neg: bool) -> F32:
    """Round an exact rational to binary32, nearest with ties to even.
    zero_neg gives the sign used when the exact value is zero."""
    if v == 0:
        return F32(Fraction(0), zero_neg)
    neg = v < 0
    a = -v if neg else v
    # exponent e with 2^e <= a < 2^(e+1)
    e = a.numerator.bit_length() - a.denominator.bit_length()
    if Fraction(2) ** e > a:
        e -= 1
    elif Fraction(2) ** (e + 1) <= a:
        e += 1
    e = max(e, _EMIN)                     # below the normal range the quantum stays fixed
    quantum = Fraction(2) ** (e - (_P - 1))
    m = a / quantum
    fl = m.numerator // m.denominator
    rem = m - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    r = fl * quantum
    if r > _MAXF:
        return F32(Fraction(0), neg, inf=True)
    if r == 0:                            # underflow to zero keeps the sign
        return F32(Fraction(0), neg)
    return F32(-r if neg else r, neg)


def _sum_zero_sign(p_val: Fraction, p_neg: bool, c: F32) -> bool:
    """Sign of an exact-zero result of p + c in round-to-nearest."""
    if p_val == 0 and c.v == 0:
        return p_neg and c.neg
    return False


def mul(a: F32, b: F32) -> F32:
    return round_binary32(a.v * b.v, a.neg != b.neg)


def add(a: F32, b: F32) -> F32:
    return round_binary32(a.v + b.v, _sum_zero_sign(a.v, a.neg, b))


def sub(a: F32, b: F32) -> F32:
    nb = F32(-b.v, not b.neg)
    return add(a, nb)


def fma(a: F32, b: F32, c: F32) -> F32:
    p = a.v * b.v
    return round_binary32(p + c.v, _sum_zero_sign(p, a.neg != b.neg, c))


def neg(a: F32) -> F32:
    return F32(-a.v, not a.neg, a.inf)


def rint(a: F32) -> F32:
    """Nearest integer, ties to even (exact: integers of binary32 size fit)."""
    fl = a.v.numerator // a.v.denominator
    rem = a.v - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return F32(Fraction(fl), a.neg if fl == 0 else None)


def c32(decimal_text: str) -> F32:
    """A decimal constant read as binary64 and then rounded to binary32."""
    return F32.from_float(struct.unpack("<f", struct.pack("<f", float(decimal_text)))[0])


# Decimal constants of Sec. II (method 1 and method 2) and of the reduction.
METHOD_DECIMALS = {
    0: dict(ss1="1.5707963235", ss2="-0.645963615", ss3="0.0796819754", ss4="-0.0046075748",
            cc1="-1.2336977925", cc2="0.2536086171", cc3="-0.0204391631"),
    1: dict(ss1="1.5707963268", ss2="-0.6466386936", ss3="0.0679105987", ss4="-0.0011573807",
            cc1="-1.2341299769", cc2="0.2465220241", cc3="-0.0123926179"),
}


def reduction_constant() -> F32:
    k = 1.0 / (2.0 * 3.1415926536)       # the division happens in binary64, as in C
    return F32.from_float(struct.unpack("<f", struct.pack("<f", k))[0])


def _madd(a, b, c, fused):
    return fma(a, b, c) if fused else add(mul(a, b), c)


def _msub_from(a, b, c, fused):
    """c - a*b."""
    return fma(neg(a), b, c) if fused else sub(c, mul(a, b))


def _series(xr: F32, sin_coef, cos_coef, fused):
    """x * (sin_coef[0] + sin_coef[1] x^2 + ...), cos_coef[0] + cos_coef[1] x^2 + ...,
    by Horner's rule in x^2, highest power first."""
    x2 = mul(xr, xr)
    t = sin_coef[-1]
    for k in reversed(sin_coef[:-1]):
        t = _madd(x2, t, k, fused)
    u = cos_coef[-1]
    for k in reversed(cos_coef[:-1]):
        u = _madd(x2, u, k, fused)
    return mul(xr, t), u


def _reduce(x: float) -> F32:
    turns = mul(F32.from_float(x), reduction_constant())
    return sub(turns, rint(turns))


def _double(s, c, fused):
    """eq. (1)."""
    return mul(F32(Fraction(2)), mul(s, c)), _msub_from(s, s, mul(c, c), fused)


def _double_eq2(s, c, fused):
    """The rejected eq. (2): cos 2u = 1 - 2 sin^2 u."""
    two = F32(Fraction(2))
    return mul(two, mul(s, c)), _msub_from(mul(two, s), s, F32(Fraction(1)), fused)


def _factor(s, c, fused, method):
    """2 - |p|^2 (method 1) or 1 / |p|^2 (method 2)."""
    if method == 0:
        return _msub_from(s, s, _msub_from(c, c, F32(Fraction(2)), fused), fused)
    d = _madd(s, s, mul(c, c), fused)
    return round_binary32(Fraction(1) / d.v, False)


def _text_factor(s, c, fused):
    """(3 - s^2 - c^2) / 2."""
    h = _msub_from(s, s, _msub_from(c, c, F32(Fraction(3)), fused), fused)
    return mul(F32(Fraction(1, 2)), h)


def _method_series(method):
    k = {n: c32(v) for n, v in METHOD_DECIMALS[method].items()}
    return ([k["ss1"], k["ss2"], k["ss3"], k["ss4"]],
            [F32(Fraction(1)), k["cc1"], k["cc2"], k["cc3"]])


def pair(x: float, fused: bool = True, method: int = 0):
    """(s, c) bits of the pair of angle x, reading of the compiled oracle."""
    s, c = _series(_reduce(x), *_method_series(method), fused)
    s, c = _double(s, c, fused)
    m = _factor(s, c, fused, method)
    s, c = _double(s, c, fused)
    return mul(s, m).bits(), mul(c, m).bits()


def variant(xr: float, fused: bool, method: int, which: str):
    """(s, c) bits of an ablation on the reduced angle xr: "no_fix", "text_fix"
    (the text's factor on the final pair) or "eq2" (both doublings with
    eq. (2), the method's factor read after the first)."""
    s, c = _series(F32.from_float(xr), *_method_series(method), fused)
    dbl = _double_eq2 if which == "eq2" else _double
    s1, c1 = dbl(s, c, fused)
    s2, c2 = dbl(s1, c1, fused)
    if which == "no_fix":
        return s2.bits(), c2.bits()
    m = _text_factor(s2, c2, fused) if which == "text_fix" else _factor(s1, c1, fused, method)
    return mul(s2, m).bits(), mul(c2, m).bits()


def pair_general(xr: float, ndoub: int, ss, cc, fused: bool, fix: bool):
    """(s, c) bits of the general ablation on the reduced angle xr: series with
    coefficients ss (sine, times x) and 1 + x^2 * cc (cosine), then ndoub
    eq. (1) doublings; with fix, the factor 2 - |p|^2 read before the last
    doubling, or (3 - |p|^2)/2 on the series pair when ndoub == 0."""
    xv = F32.from_float(xr)
    x2 = mul(xv, xv)
    t = F32.from_float(float(ss[-1]))
    for k in reversed(ss[:-1]):
        t = _madd(x2, t, F32.from_float(float(k)), fused)
    s = mul(xv, t)
    u = F32.from_float(float(cc[-1]))
    for k in reversed(cc[:-1]):
        u = _madd(x2, u, F32.from_float(float(k)), fused)
    c = _madd(x2, u, F32(Fraction(1)), fused)
    m = None
    if ndoub == 0 and fix:
        m = _text_factor(s, c, fused)
    for d in range(ndoub):
        if fix and d == ndoub - 1:
            m = _factor(s, c, fused, 0)
        s, c = _double(s, c, fused)
    if fix:
        return mul(s, m).bits(), mul(c, m).bits()
    return s.bits(), c.bits()


def pair_altivec_form(x: float, method: int = 0):
    """(s, c) bits with the multiply-adds as the AltiVec form writes them:
    products as fused multiply-adds with a +0 addend, and the negative
    multiply-subtract as -(a*b - c).  Fused arithmetic only."""
    k = {n: c32(v) for n, v in METHOD_DECIMALS[method].items()}
    zero, one, two = F32(Fraction(0), False), F32(Fraction(1)), F32(Fraction(2))

    def prod(a, b):
        return fma(a, b, zero)

    def nmsub(a, b, c):
        return neg(fma(a, b, neg(c)))

    xv = F32.from_float(x)
    x1 = prod(xv, reduction_constant())
    q1 = nmsub(rint(x1), one, x1)
    q2 = prod(q1, q1)
    t = fma(q2, fma(q2, fma(q2, k["ss4"], k["ss3"]), k["ss2"]), k["ss1"])
    s = prod(q1, t)
    c = fma(q2, fma(q2, fma(q2, k["cc3"], k["cc2"]), k["cc1"]), one)
    c2 = nmsub(s, s, prod(c, c))
    s2 = prod(two, prod(s, c))
    if method == 0:
        m = nmsub(s2, s2, nmsub(c2, c2, two))
    else:
        m = round_binary32(Fraction(1) / fma(s2, s2, prod(c2, c2)).v, False)
    c3 = nmsub(s2, s2, prod(c2, c2))
    s3 = prod(two, prod(s2, c2))
    return prod(s3, m).bits(), prod(c3, m).bits()
