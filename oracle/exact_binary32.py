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


def pair(x: float, fused: bool = True, method: int = 0):
    """(s, c) bits of the pair of angle x, reading of the compiled oracle."""
    k = {n: c32(v) for n, v in METHOD_DECIMALS[method].items()}
    one, two = F32(Fraction(1)), F32(Fraction(2))
    xv = F32.from_float(x)
    x1 = mul(xv, reduction_constant())
    q1 = sub(x1, rint(x1))
    q2 = mul(q1, q1)
    t = _madd(q2, k["ss4"], k["ss3"], fused)
    t = _madd(q2, t, k["ss2"], fused)
    t = _madd(q2, t, k["ss1"], fused)
    s = mul(q1, t)
    u = _madd(q2, k["cc3"], k["cc2"], fused)
    u = _madd(q2, u, k["cc1"], fused)
    c = _madd(q2, u, one, fused)
    pairs = []
    for _ in range(2):
        c_new = _msub_from(s, s, mul(c, c), fused)
        s_new = mul(two, mul(s, c))
        pairs.append((s_new, c_new))
        s, c = s_new, c_new
    s2, c2 = pairs[0]
    if method == 0:
        m = _msub_from(s2, s2, _msub_from(c2, c2, two, fused), fused)
    else:
        d = _madd(s2, s2, mul(c2, c2), fused)
        m = round_binary32(Fraction(1) / d.v, False)
    return mul(s, m).bits(), mul(c, m).bits()


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
