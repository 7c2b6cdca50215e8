"""The Huygens kernel's square roots (csrc/sqrt_rn.hpp) are the IEEE
correctly rounded binary32 square root on every argument they can see,
checked exhaustively on the GPU against the compiler's IEEE sqrt: sqrt_rn on
every bit pattern from 2^-96 up to +inf and on NaN, sqrt_rn_finite (the
five-instruction root of the kernel's guarded path) on every bit pattern
from 2^-96 to the largest finite binary32."""
import ctypes
import os

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "native", "libsqrt_rn_check.so")


@pytest.fixture(scope="module")
def check():
    import torch  # loads the HIP runtime torch ships before the helper library
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    assert os.path.exists(LIB), "tests/native/libsqrt_rn_check.so is not built (__graft_entry__.build())"
    L = ctypes.CDLL(LIB)
    for fn in (L.sqrt_rn_check, L.sqrt_rn_finite_check):
        fn.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                       ctypes.POINTER(ctypes.c_ulonglong), ctypes.POINTER(ctypes.c_uint32)]
        fn.restype = ctypes.c_int

    def run(lo, hi, planted=0, finite=False):
        n, first = ctypes.c_ulonglong(0), ctypes.c_uint32(0)
        fn = L.sqrt_rn_finite_check if finite else L.sqrt_rn_check
        rc = fn(lo, hi, planted, ctypes.byref(n), ctypes.byref(first))
        assert rc == 0, "HIP error %d" % rc
        return n.value, first.value
    return run


def test_every_argument_from_2_to_minus_96_to_infinity(check):
    lo = 0x0F800000          # 2^-96
    hi = 0x7F800000          # +inf
    n, first = check(lo, hi)
    assert n == 0, "%d mismatches, first at bits %08x" % (n, first)


def test_nan_zero_and_the_edge(check):
    for lo, hi in ((0x7F800001, 0x7F800001), (0x7FC00000, 0x7FC00000), (0x7FFFFFFF, 0x7FFFFFFF),
                   (0x00000000, 0x00000000)):
        n, first = check(lo, hi)
        assert n == 0, "bits %08x" % first


def test_the_check_sees_a_planted_difference(check):
    """Against the root of the next binary32 the check must count mismatches
    (about half the arguments of a binade round to a different root), so a
    check that sees nothing cannot pass."""
    lo, hi = 0x3F800000, 0x3F800000 + (1 << 20)      # [1, 1.125)
    n, first = check(lo, hi, planted=1)
    assert (hi - lo) // 4 < n < hi - lo + 1, n


def test_finite_root_on_every_argument_from_2_to_minus_96_to_the_largest_finite(check):
    n, first = check(0x0F800000, 0x7F7FFFFF, finite=True)
    assert n == 0, "%d mismatches, first at bits %08x" % (n, first)


def test_finite_root_is_not_the_ieee_root_at_infinity(check):
    """+inf gives NaN: the kernel takes sqrt_rn_finite only for arguments
    its coordinate guard keeps below 2^124."""
    n, first = check(0x7F800000, 0x7F800000, finite=True)
    assert n == 1 and first == 0x7F800000


def test_finite_root_check_sees_a_planted_difference(check):
    lo, hi = 0x3F800000, 0x3F800000 + (1 << 20)      # [1, 1.125]
    n, first = check(lo, hi, planted=1, finite=True)
    assert (hi - lo) // 4 < n <= hi - lo + 1, n
