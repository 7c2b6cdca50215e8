"""The Huygens kernel's reciprocal (rcp_rn in csrc/rcp_rn.hpp) is the IEEE
correctly rounded binary32 reciprocal on its whole range: every bit pattern
of either sign with 2^-126 <= |x| < 2^126, checked exhaustively on the GPU
against the compiler's IEEE division 1 / x.  Outside that range it is not
(which is why the kernel guards its arguments)."""
import ctypes
import os

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "native", "librcp_rn_check.so")


@pytest.fixture(scope="module")
def check():
    import torch  # loads the HIP runtime torch ships before the helper library
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    assert os.path.exists(LIB), "tests/native/librcp_rn_check.so is not built (__graft_entry__.build())"
    L = ctypes.CDLL(LIB)
    L.rcp_rn_check.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_ulonglong), ctypes.POINTER(ctypes.c_uint32)]
    L.rcp_rn_check.restype = ctypes.c_int

    def run(lo, hi, planted=0):
        n, first = ctypes.c_ulonglong(0), ctypes.c_uint32(0)
        rc = L.rcp_rn_check(lo, hi, planted, ctypes.byref(n), ctypes.byref(first))
        assert rc == 0, "HIP error %d" % rc
        return n.value, first.value
    return run


@pytest.mark.parametrize("sign", [0, 0x80000000])
def test_every_argument_from_2_to_minus_126_to_2_to_126(check, sign):
    lo = sign | 0x00800000          # 2^-126
    hi = sign | 0x7E7FFFFF          # the binary32 below 2^126
    n, first = check(lo, hi)
    assert n == 0, "%d mismatches, first at bits %08x" % (n, first)


def test_outside_the_range_it_is_not_the_ieee_reciprocal(check):
    """Subnormal x and x whose reciprocal is subnormal (or zero): the
    kernel never takes rcp_rn there."""
    n_big, _ = check(0x7E800000, 0x7F7FFFFF)         # [2^126, FLT_MAX]
    n_sub, _ = check(0x00000001, 0x007FFFFF)         # subnormals
    assert n_big > 0 and n_sub > 0


def test_the_check_sees_a_planted_difference(check):
    """Against 1 / (the next binary32) the check must count mismatches (on
    [1, 1.125) the reciprocal separates neighbouring arguments, so all of
    them), so a check that sees nothing cannot pass."""
    lo, hi = 0x3F800000, 0x3F800000 + (1 << 20)      # [1, 1.125]
    n, first = check(lo, hi, planted=1)
    assert (hi - lo) // 4 < n <= hi - lo + 1, n
    assert first == lo
