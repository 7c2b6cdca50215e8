"""Plain form on the GPU against the CPU oracle: bit-exact in FUSED and SPLIT
arithmetic (NaN compared as NaN), within the stated bound for CONTRACT."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_bit_exact, lib_loaded, log

pytestmark = pytest.mark.gpu

FUSED, SPLIT, CONTRACT = 0, 1, 2


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    return torch


def run(torch, x_host, arith=FUSED, method=0, launch=None):
    from paper_cs_0406049_amd import _capi
    x = torch.from_numpy(np.ascontiguousarray(x_host, np.float32)).cuda()
    s = torch.empty_like(x)
    c = torch.empty_like(x)
    _capi.sincos_f32_ex(x, s, c, x.numel(), arith, method, launch)
    torch.cuda.synchronize()
    return s.cpu().numpy(), c.cpu().numpy()


@pytest.mark.parametrize("method", [0, 1])
@pytest.mark.parametrize("arith", [FUSED, SPLIT])
@pytest.mark.parametrize("quarter", [0, 1, 2, 3])
def test_exhaustive_all_bit_patterns(torch_dev, arith, quarter, method):
    """Every one of the 2^32 binary32 inputs, in four quarters per mode and
    method."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    chunk = 1 << 26
    lo_q = quarter << 30
    threads = oracle.default_threads()
    xs = torch.empty(chunk, dtype=torch.float32, device="cuda")
    s = torch.empty_like(xs)
    c = torch.empty_like(xs)
    for k in range((1 << 30) // chunk):
        lo = lo_q + k * chunk
        xb = np.arange(lo, lo + chunk, dtype=np.uint64).astype(np.uint32).view(np.float32)
        xs.copy_(torch.from_numpy(xb))
        _capi.sincos_f32_ex(xs, s, c, chunk, arith, method)
        sg, cg = s.cpu().numpy(), c.cpu().numpy()
        so, co = oracle.sincos(xb, arith, method, threads=threads)
        assert_bit_exact(sg, so, "sin bits %08x.." % lo, xb)
        assert_bit_exact(cg, co, "cos bits %08x.." % lo, xb)
    log("exhaustive arith=%d method=%d quarter=%d: 2^30 inputs bit-exact" % (arith, method, quarter))


@pytest.mark.parametrize("arith", [FUSED, SPLIT])
@pytest.mark.parametrize("method", [0, 1])
def test_plain_small_workload(torch_dev, arith, method):
    from paper_cs_0406049_amd import workloads
    x = workloads.plain_small()
    sg, cg = run(torch_dev, x, arith, method)
    so, co = oracle.sincos(x, arith, method, threads=oracle.default_threads())
    assert_bit_exact(sg, so, "sin", x)
    assert_bit_exact(cg, co, "cos", x)


@pytest.mark.slow
def test_plain_roofline_workload_full(torch_dev):
    """268,435,456 angles in the benchmark's launch configuration (default
    shape), every element against the oracle, both exact modes."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, workloads
    x = workloads.plain_roofline()
    log("roofline workload generated")
    xd = torch.from_numpy(x).cuda()
    s = torch.empty_like(xd)
    c = torch.empty_like(xd)
    for arith in (FUSED, SPLIT):
        if arith == FUSED:
            _capi.sincos_f32(xd, s, c, xd.numel())
        else:
            _capi.sincos_f32_ex(xd, s, c, xd.numel(), arith, 0)
        torch.cuda.synchronize()
        so, co = oracle.sincos(x, arith, 0, threads=oracle.default_threads())
        assert_bit_exact(s.cpu().numpy(), so, "sin", x)
        assert_bit_exact(c.cpu().numpy(), co, "cos", x)
        log("roofline workload arith=%d bit-exact" % arith)


@pytest.mark.parametrize("launch", [(64, 1, 0), (256, 1, 1), (256, 2, 7), (512, 8, 0),
                                    (1024, 4, 3), (128, 4, 100)])
def test_launch_shapes(torch_dev, launch):
    x = np.random.default_rng(17).uniform(-1e3, 1e3, 1_000_003).astype(np.float32)
    sg, cg = run(torch_dev, x, FUSED, 0, launch)
    so, co = oracle.sincos(x, FUSED, 0, threads=oracle.default_threads())
    assert_bit_exact(sg, so, "sin %r" % (launch,), x)
    assert_bit_exact(cg, co, "cos %r" % (launch,), x)


CANARY = np.uint32(0x7FC0DEAD)


@pytest.mark.parametrize("offsets", [(0, 0, 0), (1, 1, 1), (2, 2, 2), (3, 3, 3), (1, 0, 0),
                                     (0, 2, 3), (3, 1, 2)])
def test_small_sizes_offsets_and_guard_bands(torch_dev, offsets):
    """n = 0..70 and n = 4099 at every 16-byte phase (head, float4 body, tail,
    and the scalar path for mismatched phases); nothing outside [0, n) of
    each output is written."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    rng = np.random.default_rng(sum(offsets))
    ox, os_, oc = offsets
    pad = 64
    for n in list(range(0, 71)) + [4099, 65536 + 5]:
        xh = rng.uniform(-50, 50, n).astype(np.float32)
        X = torch.full((n + 2 * pad,), 0, dtype=torch.float32, device="cuda")
        S = torch.from_numpy(np.full(n + 2 * pad, CANARY, np.uint32).view(np.float32)).cuda()
        C = S.clone()
        X[pad + ox:pad + ox + n] = torch.from_numpy(xh).cuda()
        xs = X[pad + ox:pad + ox + n]
        ss = S[pad + os_:pad + os_ + n]
        cs = C[pad + oc:pad + oc + n]
        _capi.sincos_f32(xs.data_ptr(), ss.data_ptr(), cs.data_ptr(), n)
        torch.cuda.synchronize()
        Sh = S.cpu().numpy().view(np.uint32)
        Ch = C.cpu().numpy().view(np.uint32)
        so, co = oracle.sincos(xh, FUSED, 0)
        assert_bit_exact(Sh[pad + os_:pad + os_ + n].view(np.float32), so, "sin n=%d" % n, xh)
        assert_bit_exact(Ch[pad + oc:pad + oc + n].view(np.float32), co, "cos n=%d" % n, xh)
        for arr, o in ((Sh, os_), (Ch, oc)):
            assert np.all(arr[:pad + o] == CANARY) and np.all(arr[pad + o + n:] == CANARY), n


def test_in_place(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    xh = np.random.default_rng(5).uniform(-1e4, 1e4, 1 << 20).astype(np.float32)
    so, co = oracle.sincos(xh, FUSED, 0, threads=oracle.default_threads())
    x = torch.from_numpy(xh).cuda()
    c = torch.empty_like(x)
    _capi.sincos_f32(x, x, c, x.numel())          # s overwrites x
    torch.cuda.synchronize()
    assert_bit_exact(x.cpu().numpy(), so, "sin in place")
    assert_bit_exact(c.cpu().numpy(), co, "cos")
    x = torch.from_numpy(xh).cuda()
    s = torch.empty_like(x)
    _capi.sincos_f32(x, s, x, x.numel())          # c overwrites x
    torch.cuda.synchronize()
    assert_bit_exact(s.cpu().numpy(), so, "sin")
    assert_bit_exact(x.cpu().numpy(), co, "cos in place")


def test_special_values(torch_dev):
    x = np.array([np.inf, -np.inf, np.nan, 0.0, -0.0, 1e-45, -1e-45, 1e-40, 1.17549435e-38,
                  3.4028235e38, -3.4028235e38, 5.27e7, 6e7, math.pi, -math.pi, math.pi / 2,
                  math.pi / 4, 0.5 / (1 / (2 * math.pi))], np.float32)
    for arith in (FUSED, SPLIT):
        for method in (0, 1):
            sg, cg = run(torch_dev, x, arith, method)
            so, co = oracle.sincos(x, arith, method)
            assert_bit_exact(sg, so, "sin", x)
            assert_bit_exact(cg, co, "cos", x)


@pytest.mark.parametrize("method", [0, 1])
def test_contract_mode_within_stated_bound(torch_dev, method):
    """With contraction allowed the compiler may fuse any product into the sum
    that consumes it.  Two reduced angles are then possible: the rounded
    x1 = fl(x*K) less rint(x1) (exact), or x*K fused into that subtraction,
    one rounding of the exact x*K - rint(x1).  x*K is exact in binary64
    (24-bit by 24-bit significands), so the second is float32(x*K - r) with
    the product taken in double.  Every other fusion (in the series, the
    doublings and the factor) moves a component by less than 2^-20.  So each
    GPU pair lies within 2^-20, in both components, of the SPLIT oracle's pair
    of one of the two reduced angles: a bound that does not grow with |x|."""
    x = np.concatenate([
        np.random.default_rng(8).uniform(-8 * math.pi, 8 * math.pi, 1 << 20),
        np.random.default_rng(9).uniform(-1e4, 1e4, 1 << 20),
        np.random.default_rng(10).uniform(-0.5, 0.5, 1 << 18)]).astype(np.float32)
    sg, cg = run(torch_dev, x, CONTRACT, method)
    k = np.float32(1.0 / (2.0 * 3.1415926536))
    x1 = (x * k).astype(np.float32)
    r = np.rint(x1)
    q_split = (x1 - r).astype(np.float32)
    q_fused = (x.astype(np.float64) * np.float64(k) - r.astype(np.float64)).astype(np.float32)
    thr = oracle.default_threads()
    bound = 2.0 ** -20
    ok = np.zeros(x.size, bool)
    worst = np.full(x.size, np.inf)
    for q in (q_split, q_fused):
        so, co = oracle.pair_from_reduced(q, SPLIT, method, threads=thr)
        d = np.maximum(np.abs(sg.astype(np.float64) - so), np.abs(cg.astype(np.float64) - co))
        ok |= d <= bound
        worst = np.minimum(worst, d)
    log("contract vs split: max deviation from the nearer reduction %.3g; fused reduction "
        "differs on %.2f%% of inputs" % (worst.max(), 100 * np.mean(q_split != q_fused)))
    assert ok.all(), x[~ok][:10]


def test_gpu_accuracy_matches_paper(torch_dev):
    """The GPU pairs themselves reproduce the printed RMS error (uniform angles
    in [-pi, pi) against the double library)."""
    x = np.random.default_rng(7).uniform(-math.pi, math.pi, 1 << 22).astype(np.float32)
    sg, cg = run(torch_dev, x, FUSED, 0)
    xd = x.astype(np.float64)
    e = np.sqrt((sg - np.sin(xd)) ** 2 + (cg - np.cos(xd)) ** 2)
    rms = float(np.sqrt(np.mean(e ** 2)))
    log("GPU RMS vector error %.3g (paper 1.2e-7), max %.3g" % (rms, e.max()))
    assert abs(rms / 1.2e-7 - 1) < 0.05


@pytest.mark.parametrize("layout", [0, 1])
def test_interleaved_layouts(torch_dev, layout):
    """complex64 (cos, sin) pairs, and the paper's blocks of 4 sines then 4
    cosines: the same bits as the SoA pairs, nothing written past the end."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    rng = np.random.default_rng(30 + layout)
    for n in list(range(0, 21)) + [255, 256, 257, 1023, 1_000_003, 1 << 22]:
        xh = rng.uniform(-1e3, 1e3, n).astype(np.float32)
        so, co = oracle.sincos(xh, FUSED, 0, threads=oracle.default_threads())
        out_len = 2 * n if layout == 0 else 8 * ((n + 3) // 4)
        x = torch.from_numpy(xh).cuda() if n else torch.empty(0, device="cuda")
        out = torch.from_numpy(np.full(out_len + 64, CANARY, np.uint32).view(np.float32)).cuda()
        _capi.sincos_f32_interleaved(x, out, n, layout)
        torch.cuda.synchronize()
        oh = out.cpu().numpy()
        if layout == 0:
            assert_bit_exact(oh[0:2 * n:2], co, "cos n=%d" % n, xh)
            assert_bit_exact(oh[1:2 * n:2], so, "sin n=%d" % n, xh)
        else:
            nb = (n + 3) // 4
            blocks = oh[:8 * nb].reshape(nb, 8) if nb else np.zeros((0, 8), np.float32)
            sp = np.full(4 * nb, np.nan, np.float32)
            cp = np.full(4 * nb, np.nan, np.float32)
            sp[:n], cp[:n] = so, co
            for b in range(nb):
                m = min(4, n - 4 * b)
                assert np.array_equal(blocks[b, :m].view(np.uint32), sp[4 * b:4 * b + m].view(np.uint32)), (n, b)
                assert np.array_equal(blocks[b, 4:4 + m].view(np.uint32), cp[4 * b:4 * b + m].view(np.uint32)), (n, b)
        assert np.all(oh[out_len:].view(np.uint32) == CANARY), n


def _pair_ceiling_reference(xh, reps):
    """The ceiling kernel's sums written out with the oracle's pair and binary32
    adds: 8 chains theta_r = x + r, +1 per step, sines and cosines summed in
    step order, then sum over r of (sines_r + cosines_r)."""
    one = np.float32(1.0)
    th = [(xh + np.float32(r)).astype(np.float32) for r in range(8)]
    ss = [np.zeros_like(xh) for _ in range(8)]
    cs = [np.zeros_like(xh) for _ in range(8)]
    for _ in range(reps):
        for r in range(8):
            s, c = oracle.sincos(th[r], FUSED, 0)
            ss[r] = (ss[r] + s).astype(np.float32)
            cs[r] = (cs[r] + c).astype(np.float32)
            th[r] = (th[r] + one).astype(np.float32)
    o = np.zeros_like(xh)
    for r in range(8):
        o = (o + (ss[r] + cs[r]).astype(np.float32)).astype(np.float32)
    return o


@pytest.mark.parametrize("n,reps", [(1, 1), (777, 3), (4096, 2), (65537, 1), (300, 0)])
def test_pair_ceiling_kernel_matches_its_definition(torch_dev, n, reps):
    """The VALU-ceiling measurement kernel computes what its header says (its
    pairs are the method's, bit for bit)."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    xh = np.random.default_rng(n).uniform(-50, 50, n).astype(np.float32)
    x = torch.from_numpy(xh).cuda()
    out = torch.from_numpy(np.full(n + 64, CANARY, np.uint32).view(np.float32)).cuda()
    _capi.sincos_pair_ceiling_f32(x, out, n, reps)
    torch.cuda.synchronize()
    oh = out.cpu().numpy()
    assert_bit_exact(oh[:n], _pair_ceiling_reference(xh, reps), "pair ceiling n=%d" % n, xh)
    assert np.all(oh[n:].view(np.uint32) == CANARY)


def test_binding_rejects_short_arrays(torch_dev):
    """The binding checks that every tensor holds what the call will touch,
    before anything reaches the device."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    x = torch.zeros(100, device="cuda")
    short = torch.zeros(99, device="cuda")
    ok = torch.zeros(100, device="cuda")
    with pytest.raises(ValueError):
        _capi.sincos_f32(x, short, ok)
    with pytest.raises(ValueError):
        _capi.sincos_f32(x, ok, ok.clone(), n=101)
    with pytest.raises(ValueError):
        _capi.sincos_f32_interleaved(x, torch.zeros(199, device="cuda"), layout=0)
    with pytest.raises(ValueError):
        _capi.sincos_f32_interleaved(x[:5], torch.zeros(15, device="cuda"), layout=1)
    with pytest.raises(ValueError):
        _capi.sincos_f32_backward(x, ok, short, None, ok.clone())
    with pytest.raises(ValueError):
        _capi.sincos_f32_ragged([(x, ok, short)], [100])
    with pytest.raises(ValueError):
        _capi.huygens_f32(x, ok, torch.zeros(7, device="cuda"), 1.0, 10.0, ok.clone(), ok.clone(),
                          S=2)
    torch.cuda.synchronize()
