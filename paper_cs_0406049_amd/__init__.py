"""MI355X (gfx950) implementation of Mendenhall's branch-free single-precision
sine-cosine pair (2004): HIP kernels behind a C ABI (include/sincos.h), with a
thin ctypes binding.  PyTorch supplies device memory and streams only.

    from paper_cs_0406049_amd import sincos
    s, c = sincos(x)            # x: float32 tensor on the GPU

Submodules: ``_capi`` (the binding, same names as the C ABI), ``autograd``
(torch.autograd.Functions over the adjoint kernels), ``autotune`` (launch-shape
search for the ragged form), ``serve`` (the request server), ``workloads``
(seeded synthetic inputs), ``build`` (hipcc build of the library).
"""
from __future__ import annotations

__all__ = ["sincos", "sincos_backward", "version"]

ARITH_FUSED, ARITH_SPLIT, ARITH_CONTRACT = 0, 1, 2
METHOD_NORMALIZED, METHOD_ARCTAN = 0, 1


def sincos(x, arith: int = ARITH_FUSED, method: int = METHOD_NORMALIZED, launch=None,
           stream=None):
    """(s, c) of a float32 GPU tensor x, new tensors of x's shape."""
    import torch
    from . import _capi
    if x.dtype != torch.float32 or not x.is_cuda:
        raise ValueError("x must be a float32 tensor on the GPU")
    x = x.contiguous()
    s = torch.empty_like(x)
    c = torch.empty_like(x)
    _capi.sincos_f32_ex(x, s, c, x.numel(), arith, method, launch, stream)
    return s, c


def sincos_backward(s, c, gs=None, gc=None, stream=None):
    """gx = gs*c - gc*s (None counts as zero)."""
    import torch
    from . import _capi
    gx = torch.empty_like(s)
    _capi.sincos_f32_backward(s, c, gs, gc, gx, s.numel(), stream)
    return gx


def version() -> str:
    from . import _capi
    return _capi.version()
