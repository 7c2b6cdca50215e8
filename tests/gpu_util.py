"""Helpers shared by the GPU tests (comparison, device buffers)."""
import numpy as np


def lib_loaded():
    """The HIP library, loaded; GPU tests fail (not skip) if it is missing."""
    from paper_cs_0406049_amd import _capi
    return _capi.lib()


def bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def same_bits_nan_equal(a, b):
    """Bitwise equality, with any NaN equal to any NaN (payloads may differ)."""
    a = np.ascontiguousarray(a, np.float32)
    b = np.ascontiguousarray(b, np.float32)
    eq = bits(a) == bits(b)
    both_nan = np.isnan(a) & np.isnan(b)
    return eq | both_nan


def assert_bit_exact(got, want, what="", x=None):
    ok = same_bits_nan_equal(got, want)
    if not ok.all():
        i = int(np.flatnonzero(~ok)[0])
        extra = "" if x is None else " at x=%r (bits %08x)" % (float(x[i]), int(bits(x[i:i + 1])[0]))
        raise AssertionError("%s: %d of %d elements differ; first index %d: got %r want %r%s" % (
            what, int((~ok).sum()), ok.size, i, float(got[i]), float(want[i]), extra))


def log(msg):
    print(msg, flush=True)


class _DeviceArray:
    """Exposes a device address as a float32 array (CUDA array interface)."""

    def __init__(self, ptr, n):
        self.__cuda_array_interface__ = {"shape": (int(n),), "typestr": "<f4",
                                         "data": (int(ptr), False), "version": 2}


def device_view(torch, ptr, n):
    """A float32 tensor aliasing n elements at a device address."""
    return torch.as_tensor(_DeviceArray(ptr, n), device="cuda")
