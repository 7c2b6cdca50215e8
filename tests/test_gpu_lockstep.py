"""The pair arithmetic on N-element vectors (csrc/sincos_core.hpp, fvec<N>:
N pairs per lane in lockstep, as the Huygens kernel evaluates a group of
sources) gives each element exactly the bits of the same arithmetic on one
float: every binary32 bit pattern, widths 2 and 4, both methods, fused and
split arithmetic, checked exhaustively on the GPU."""
import ctypes
import os

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "native", "liblockstep_check.so")


@pytest.fixture(scope="module")
def check():
    import torch  # loads the HIP runtime torch ships before the helper library
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    assert os.path.exists(LIB), "tests/native/liblockstep_check.so is not built (__graft_entry__.build())"
    L = ctypes.CDLL(LIB)
    L.lockstep_check.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint32,
                                 ctypes.c_uint32, ctypes.c_int,
                                 ctypes.POINTER(ctypes.c_ulonglong),
                                 ctypes.POINTER(ctypes.c_uint32)]
    L.lockstep_check.restype = ctypes.c_int

    def run(width, arith, method, lo, hi, planted=0):
        n, first = ctypes.c_ulonglong(0), ctypes.c_uint32(0)
        rc = L.lockstep_check(width, arith, method, lo, hi, planted, ctypes.byref(n),
                              ctypes.byref(first))
        assert rc == 0, "HIP error %d" % rc
        return n.value, first.value
    return run


@pytest.mark.parametrize("method", [0, 1], ids=["first", "second"])
@pytest.mark.parametrize("arith", [0, 1], ids=["fused", "split"])
@pytest.mark.parametrize("width", [2, 4])
def test_every_bit_pattern_matches_the_scalar_pair(check, width, arith, method):
    n, first = check(width, arith, method, 0, 0xFFFFFFFF)
    assert n == 0, "%d mismatches, first at bits %08x" % (n, first)


def test_the_check_sees_a_planted_difference(check):
    """Against the scalar pair of the next bit pattern the check must count
    mismatches (on [1, 2) neighbouring angles give different pairs), so a
    check that sees nothing cannot pass."""
    lo, hi = 0x3F800000, 0x3F800000 + (1 << 16)
    n, first = check(2, 0, 0, lo, hi, planted=1)
    assert (hi - lo) // 2 < n <= hi - lo + 1, n
    assert first == lo


def test_bad_arguments_are_rejected(check):
    L = ctypes.CDLL(LIB)
    n, first = ctypes.c_ulonglong(0), ctypes.c_uint32(0)
    assert L.lockstep_check(3, 0, 0, 0, 1, 0, ctypes.byref(n), ctypes.byref(first)) != 0
    assert L.lockstep_check(2, 0, 0, 5, 1, 0, ctypes.byref(n), ctypes.byref(first)) != 0
