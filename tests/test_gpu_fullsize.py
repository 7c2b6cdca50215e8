"""Forms at the sizes bench.py times them, in the same launch configuration:
the elementwise adjoint over 2^28 elements and the interleaved layouts over
the 268M-angle roofline workload (every output against the oracle), and the
ablation kernels over the roofline workload (sampled outputs: both ends, the
tail, and 200,000 random positions)."""
import numpy as np
import pytest

import oracle
from paper_cs_0406049_amd.workloads import taylor_series
from gpu_util import assert_bit_exact, lib_loaded, log

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    return torch


@pytest.fixture(scope="module")
def roofline(torch_dev):
    from paper_cs_0406049_amd import workloads
    xh = workloads.plain_roofline()
    return xh, torch_dev.from_numpy(xh).cuda()


def _sample(n, seed):
    rng = np.random.default_rng(seed)
    return np.unique(np.concatenate([np.arange(0, 1000), np.arange(n - 1000, n),
                                     rng.integers(0, n, 200_000)])).astype(np.int64)


def test_adjoint_full_size(torch_dev):
    """gx = gs*c - gc*s over 2^28 elements with both gradients, inputs drawn
    as the bench draws them (uniform [0, 1) on the device)."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    n = 1 << 28
    g = torch.Generator(device="cuda").manual_seed(5)
    s_ = torch.rand(n, device="cuda", generator=g)
    c_ = torch.rand(n, device="cuda", generator=g)
    gs = torch.rand(n, device="cuda", generator=g)
    gc = torch.rand(n, device="cuda", generator=g)
    gx = torch.empty_like(s_)
    _capi.sincos_f32_backward(s_, c_, gs, gc, gx, n)
    torch.cuda.synchronize()
    want = oracle.sincos_backward(s_.cpu().numpy(), c_.cpu().numpy(), gs.cpu().numpy(),
                                  gc.cpu().numpy())
    assert_bit_exact(gx.cpu().numpy(), want, "adjoint 2^28")
    log("adjoint: 2^28 outputs bit-exact")


@pytest.mark.parametrize("layout", [0, 1])
def test_interleaved_roofline_workload(torch_dev, roofline, layout):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    xh, x = roofline
    out = torch.empty(2 * x.numel(), device="cuda")
    _capi.sincos_f32_interleaved(x, out, x.numel(), layout)
    torch.cuda.synchronize()
    so, co = oracle.sincos(xh, 0, 0, threads=oracle.default_threads())
    o = out.cpu().numpy()
    if layout == 0:
        assert_bit_exact(o[0::2], co, "complex64 cos", xh)
        assert_bit_exact(o[1::2], so, "complex64 sin", xh)
    else:
        blocks = o.reshape(-1, 8)
        assert_bit_exact(blocks[:, :4].reshape(-1), so, "phase blocks sin", xh)
        assert_bit_exact(blocks[:, 4:].reshape(-1), co, "phase blocks cos", xh)


@pytest.mark.parametrize("case", ["no_fix", "text_fix", "eq2", "doublings_0", "doublings_5"])
def test_ablations_roofline_workload_sampled(torch_dev, roofline, case):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    xh, x = roofline
    n = x.numel()
    s = torch.empty_like(x)
    c = torch.empty_like(x)
    if case.startswith("doublings"):
        nd = int(case.split("_")[1])
        ss, cc = taylor_series(nd, *{0: (6, 6), 5: (2, 2)}[nd])
        _capi.sincos_f32_doublings(x, s, c, nd, ss, cc, n)
        idx = _sample(n, nd)
        so, co = oracle.sincos_general(xh[idx], nd, ss, cc)
    else:
        v = {"no_fix": 1, "text_fix": 2, "eq2": 3}[case]
        _capi.sincos_f32_variant(x, s, c, n, variant=v)
        idx = _sample(n, v)
        so, co = oracle.sincos_variant(xh[idx], 0, 0, v)
    torch.cuda.synchronize()
    ti = torch.from_numpy(idx).cuda()
    assert_bit_exact(s.index_select(0, ti).cpu().numpy(), so, case + " sin", xh[idx])
    assert_bit_exact(c.index_select(0, ti).cpu().numpy(), co, case + " cos", xh[idx])
