"""torch.autograd.Functions over the library's forward and adjoint kernels.

SinCosFn:   x -> (s, c); backward gx = gs*c - gc*s (the analytic derivative of
            the pair, evaluated with the approximated pair; the method is
            smooth away from the wrap at odd multiples of pi, which is what
            makes this usable in fitting).
SinusoidFn: (t, A, w, phi) -> y, y_i = sum_k A_k sin(w_k t_i + phi_k);
            backward gives dL/dA, dL/dw, dL/dphi from dL/dy (one adjoint
            kernel plus a deterministic reduction).  dL/dt is not provided.

All arithmetic runs in the HIP kernels; these classes allocate outputs and
marshal arguments.
"""
from __future__ import annotations

import torch

from . import _capi


def _f32_gpu(name, a):
    if not (a.is_cuda and a.dtype == torch.float32):
        raise ValueError("%s must be a float32 tensor on the GPU" % name)
    return a.contiguous()


class SinCosFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, arith: int = _capi.ARITH_FUSED, method: int = _capi.METHOD_NORMALIZED):
        x = _f32_gpu("x", x)
        s = torch.empty_like(x)
        c = torch.empty_like(x)
        _capi.sincos_f32_ex(x, s, c, x.numel(), arith, method)
        ctx.save_for_backward(s, c)
        return s, c

    @staticmethod
    def backward(ctx, gs, gc):
        s, c = ctx.saved_tensors
        gs = None if gs is None else gs.contiguous()
        gc = None if gc is None else gc.contiguous()
        gx = torch.empty_like(s)
        _capi.sincos_f32_backward(s, c, gs, gc, gx, s.numel())
        return gx, None, None


def sincos(x, arith: int = _capi.ARITH_FUSED, method: int = _capi.METHOD_NORMALIZED):
    """Differentiable (s, c) of x."""
    return SinCosFn.apply(x, arith, method)


class SinusoidFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, t, A, w, phi):
        t = _f32_gpu("t", t)
        A, w, phi = _f32_gpu("A", A), _f32_gpu("w", w), _f32_gpu("phi", phi)
        if not (A.numel() == w.numel() == phi.numel()):
            raise ValueError("A, w and phi must have the same length")
        y = torch.empty_like(t)
        _capi.sinusoid_f32_forward(t, A, w, phi, y, t.numel(), A.numel())
        ctx.save_for_backward(t, A, w, phi)
        return y

    @staticmethod
    def backward(ctx, gy):
        t, A, w, phi = ctx.saved_tensors
        if ctx.needs_input_grad[0]:
            raise NotImplementedError("SinusoidFn gives no gradient with respect to t")
        gy = gy.contiguous()
        N, K = t.numel(), A.numel()
        gA = torch.empty_like(A)
        gw = torch.empty_like(w)
        gphi = torch.empty_like(phi)
        nbytes = _capi.sinusoid_f32_backward_workspace_bytes(N, K)
        ws = torch.empty(max(nbytes, 4), dtype=torch.uint8, device=t.device)
        _capi.sinusoid_f32_backward(t, gy, A, w, phi, gA, gw, gphi, ws, nbytes, N, K)
        return None, gA, gw, gphi


def sinusoid(t, A, w, phi):
    """Differentiable y(t) = sum_k A_k sin(w_k t + phi_k)."""
    return SinusoidFn.apply(t, A, w, phi)


def sinusoid_loss_and_grads(t, y_obs, A, w, phi):
    """L = 1/2 sum (y - y_obs)^2 and (dL/dA, dL/dw, dL/dphi) via the kernels,
    without autograd bookkeeping: one pass over the samples (forward model,
    residual kept on chip, adjoint sums), then one reduction.  L is a 0-dim
    float32 tensor; the gradients are the same bits as the forward kernel's
    residual followed by the adjoint kernel."""
    N, K = t.numel(), A.numel()
    loss = torch.empty(1, dtype=torch.float32, device=t.device)
    gA = torch.empty_like(A)
    gw = torch.empty_like(w)
    gphi = torch.empty_like(phi)
    nb = _capi.sinusoid_f32_fit_step_workspace_bytes(N, K)
    ws = torch.empty(max(nb, 4), dtype=torch.uint8, device=t.device)
    _capi.sinusoid_f32_fit_step(t, y_obs, A, w, phi, loss, gA, gw, gphi, ws, nb, N, K)
    return loss[0], gA, gw, gphi


def sinusoid_loss_and_grads_two_pass(t, y_obs, A, w, phi):
    """The same step as two library calls: the forward kernel fused with the
    residual and the loss, then the adjoint kernel over the stored residual."""
    N, K = t.numel(), A.numel()
    r = torch.empty_like(t)
    loss = torch.empty(1, dtype=torch.float32, device=t.device)
    gA = torch.empty_like(A)
    gw = torch.empty_like(w)
    gphi = torch.empty_like(phi)
    nb_fwd = _capi.sinusoid_f32_residual_workspace_bytes(N)
    nb_adj = _capi.sinusoid_f32_backward_workspace_bytes(N, K)
    ws = torch.empty(max(nb_fwd, nb_adj, 4), dtype=torch.uint8, device=t.device)
    _capi.sinusoid_f32_residual(t, y_obs, A, w, phi, r, loss, ws, nb_fwd, N, K)
    _capi.sinusoid_f32_backward(t, r, A, w, phi, gA, gw, gphi, ws, nb_adj, N, K)
    return loss[0], gA, gw, gphi
