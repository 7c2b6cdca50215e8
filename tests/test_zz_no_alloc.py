"""The allocation-free fit step (sinusoid_f32_fit_step_noalloc): its partials
live in the library's static device scratch instead of a caller workspace.
Through the C ABI it gives the same loss and gradient bits as
sinusoid_f32_fit_step on consecutive calls whose sizes shrink (the scratch
keeps the previous call's partials), and the host rejects sizes beyond the
scratch before any device work."""
import math

import numpy as np
import pytest

from paper_cs_0406049_amd import _capi, build as hipbuild

SCRATCH = _capi.FIT_SCRATCH_BYTES
BASE = 1 << 32       # fake device addresses, never dereferenced (host checks fail first)


def _problem(N, K, seed):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0, 1000, N).astype(np.float32)
    A = rng.standard_normal(K).astype(np.float32)
    w = rng.uniform(0.1, 10, K).astype(np.float32)
    phi = rng.uniform(-math.pi, math.pi, K).astype(np.float32)
    y_obs = rng.standard_normal(N).astype(np.float32)
    return t, y_obs, A, w, phi


def _max_samples(K):
    """Largest N whose partials fit the scratch at K frequencies."""
    per_part = (3 * 64 * -(-K // 64) + 1) * 4
    return (SCRATCH // per_part) * 2048


def test_scratch_limit_rejected_on_the_host():
    if not hipbuild.is_built():
        hipbuild.build()
    L = _capi.lib()
    f = L.sinusoid_f32_fit_step_noalloc
    t, yo, A, w, p = (BASE + k * (1 << 30) for k in range(5))
    loss, gA, gw, gp = (BASE + (5 << 30) + k * 65536 for k in range(4))
    for K in (1, 64, 65, 130):
        nmax = _max_samples(K)
        assert L.sinusoid_f32_fit_step_workspace_bytes(nmax, K) <= SCRATCH
        assert L.sinusoid_f32_fit_step_workspace_bytes(nmax + 1, K) > SCRATCH
        rc = f(t, yo, nmax + 1, A, w, p, K, loss, gA, gw, gp, None)
        assert rc == _capi.EINVAL and "scratch" in _capi.last_error(), (K, _capi.last_error())
    assert _max_samples(64) == 22_253_568          # the limit sincos.h states
    assert f(t, yo, -1, A, w, p, 8, loss, gA, gw, gp, None) == _capi.EINVAL
    assert f(t, yo, 16, A, w, p, 8, None, gA, gw, gp, None) == _capi.EINVAL
    assert f(t, yo, 16, A, w, p, 8, loss, A, gw, gp, None) == _capi.EOVERLAP
    assert f(t, yo, 16, A, w, p, 8, loss, gA, gw, gp + 2, None) == _capi.EINVAL


@pytest.mark.gpu
def test_noalloc_fit_step_matches_the_workspace_entry_point():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    _capi.lib()
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda() if a.size else \
        torch.empty(0, device="cuda")  # noqa: E731
    # large, then smaller (fewer partials, another frequency padding, so the
    # loss partials sit at another offset), then the largest size the
    # scratch holds, then a small one again, then an empty one
    cases = [(3_000_000, 64), (5000, 130), (_max_samples(64), 64), (2049, 3), (0, 5)]
    for idx, (N, K) in enumerate(cases):
        print("noalloc fit step: call %d, N=%d K=%d" % (idx, N, K), flush=True)
        t, y_obs, A, w, phi = _problem(N, K, 100 + idx)
        args = [d(t), d(y_obs), d(A), d(w), d(phi)]
        Kk = max(K, 1)
        out_ws = [torch.full((1,), float("nan"), device="cuda")] + \
            [torch.full((Kk,), float("nan"), device="cuda") for _ in range(3)]
        out_na = [torch.full((1,), float("nan"), device="cuda")] + \
            [torch.full((Kk,), float("nan"), device="cuda") for _ in range(3)]
        nb = _capi.sinusoid_f32_fit_step_workspace_bytes(N, K)
        assert nb <= SCRATCH
        ws = torch.empty(max(nb, 4), dtype=torch.uint8, device="cuda")
        _capi.sinusoid_f32_fit_step(*args, *out_ws, ws, nb, N=N, K=K)
        _capi.sinusoid_f32_fit_step_noalloc(*args, *out_na, N=N, K=K)
        torch.cuda.synchronize()
        for name, a, b in zip(("loss", "gA", "gw", "gphi"), out_ws, out_na):
            n = 1 if name == "loss" else K
            a, b = a[:n].cpu().numpy(), b[:n].cpu().numpy()
            assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), (idx, N, K, name)
            assert np.all(np.isfinite(b)), (idx, N, K, name)
        if N == 0:
            assert float(out_na[0].cpu()[0]) == 0.0
        del args, ws
