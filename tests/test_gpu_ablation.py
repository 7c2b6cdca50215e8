"""The Sec. II ablations on the GPU (sincos_f32_variant, sincos_f32_doublings)
against the oracle's ablations, bit for bit: the method's alternatives (no
fix, the text's fix, the eq. (2) doubling) in both arithmetics and methods,
and the general form with n = 0..5 doublings after Taylor series, with and
without the fix.  The listing variant and the general form with n = 2, the
printed series and the fix give the plain form's bits."""
import numpy as np
import pytest

import oracle
from paper_cs_0406049_amd.workloads import taylor_series
from gpu_util import assert_bit_exact, lib_loaded

pytestmark = pytest.mark.gpu

# series lengths per doubling count (the ablation's table)
TERMS = {0: (6, 6), 1: (5, 4), 2: (4, 3), 3: (3, 3), 4: (3, 2), 5: (2, 2)}


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    return torch


@pytest.fixture(scope="module")
def angles(torch_dev):
    """U[-8 pi, 8 pi) plus specials, subnormals, exact half turns, large
    angles, and a length that leaves a 3-element tail."""
    rng = np.random.default_rng(21)
    x = rng.uniform(-8 * np.pi, 8 * np.pi, (1 << 20) - 5).astype(np.float32)
    extra = np.array([0.0, -0.0, 1e-40, -1e-40, np.inf, -np.inf, np.nan, np.pi, -np.pi,
                      np.float32(0.5) / np.float32(0.15915494), 6e7, -3e8, 1e4, 1e-3],
                     np.float32)
    x = np.concatenate([x, extra])
    assert x.size % 4 == 1
    return x, torch_dev.from_numpy(x).cuda()


def _run(torch, fn, xd):
    s = torch.empty_like(xd)
    c = torch.empty_like(xd)
    fn(xd, s, c)
    torch.cuda.synchronize()
    return s.cpu().numpy(), c.cpu().numpy()


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("arith", [0, 1])
def test_variants_bit_exact(torch_dev, angles, arith, method, variant):
    from paper_cs_0406049_amd import _capi
    x, xd = angles
    s, c = _run(torch_dev, lambda a, b, d: _capi.sincos_f32_variant(a, b, d, arith=arith,
                                                                    method=method,
                                                                    variant=variant), xd)
    so, co = oracle.sincos_variant(x, arith, method, variant, threads=oracle.default_threads())
    what = "variant %d arith %d method %d" % (variant, arith, method)
    assert_bit_exact(s, so, what + " sin", x)
    assert_bit_exact(c, co, what + " cos", x)
    if variant == 0:   # the listing variant is the plain form
        sp, cp = _run(torch_dev, lambda a, b, d: _capi.sincos_f32_ex(a, b, d, arith=arith,
                                                                     method=method), xd)
        assert_bit_exact(s, sp, what + " vs plain sin", x)
        assert_bit_exact(c, cp, what + " vs plain cos", x)


@pytest.mark.parametrize("fix", [True, False])
@pytest.mark.parametrize("ndoub", sorted(TERMS))
@pytest.mark.parametrize("arith", [0, 1])
def test_doublings_bit_exact(torch_dev, angles, arith, ndoub, fix):
    from paper_cs_0406049_amd import _capi
    x, xd = angles
    ss, cc = taylor_series(ndoub, *TERMS[ndoub])
    s, c = _run(torch_dev, lambda a, b, d: _capi.sincos_f32_doublings(a, b, d, ndoub, ss, cc,
                                                                      arith=arith, fix=fix), xd)
    so, co = oracle.sincos_general(x, ndoub, ss, cc, arith, fix=fix,
                                   threads=oracle.default_threads())
    what = "doublings n=%d arith %d fix %d" % (ndoub, arith, fix)
    assert_bit_exact(s, so, what + " sin", x)
    assert_bit_exact(c, co, what + " cos", x)


@pytest.mark.parametrize("arith", [0, 1])
def test_doublings_with_printed_series_are_the_method(torch_dev, angles, arith):
    from paper_cs_0406049_amd import _capi
    x, xd = angles
    k = oracle.constants(oracle.METHOD1)
    s, c = _run(torch_dev, lambda a, b, d: _capi.sincos_f32_doublings(a, b, d, 2, k[1:5], k[5:8],
                                                                      arith=arith), xd)
    sp, cp = _run(torch_dev, lambda a, b, d: _capi.sincos_f32_ex(a, b, d, arith=arith), xd)
    assert_bit_exact(s, sp, "n=2 printed series sin", x)
    assert_bit_exact(c, cp, "n=2 printed series cos", x)


def test_tails_and_in_place(torch_dev):
    """Every length 0..9 (the float4 body and the scalar tail), and x == s."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    rng = np.random.default_rng(5)
    ss, cc = taylor_series(3, 3, 3)
    for n in range(10):
        xh = rng.uniform(-50, 50, n).astype(np.float32)
        for variant in (1, 3):
            xd = torch.from_numpy(xh).cuda() if n else torch.empty(0, device="cuda")
            c = torch.empty_like(xd)
            _capi.sincos_f32_variant(xd, xd, c, n=n, variant=variant)   # in place over x
            torch.cuda.synchronize()
            so, co = oracle.sincos_variant(xh, 0, 0, variant)
            assert_bit_exact(xd.cpu().numpy(), so, "in place n=%d" % n)
            assert_bit_exact(c.cpu().numpy(), co, "in place cos n=%d" % n)
        xd = torch.from_numpy(xh).cuda() if n else torch.empty(0, device="cuda")
        s, c = torch.empty_like(xd), torch.empty_like(xd)
        _capi.sincos_f32_doublings(xd, s, c, 3, ss, cc, n=n)
        torch.cuda.synchronize()
        so, co = oracle.sincos_general(xh, 3, ss, cc)
        assert_bit_exact(s.cpu().numpy(), so, "doublings n=%d" % n)
        assert_bit_exact(c.cpu().numpy(), co, "doublings cos n=%d" % n)
