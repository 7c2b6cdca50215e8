"""Huygens point-source sum on the GPU: bit-exact against the oracle (the
binary32 sequence: four blocks of sources each summed in order, IEEE square
root, both quotients from one IEEE reciprocal), on the fast paths
(sqrt_rn, rcp_rn) and on the IEEE fallbacks the kernel takes for extreme
screen distances and coordinates."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_bit_exact, lib_loaded, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    return torch


def run(torch, xo, yo, src, k, L):
    from paper_cs_0406049_amd import _capi
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()  # noqa: E731
    xd, yd, sd = d(xo), d(yo), d(src.reshape(-1))
    re = torch.empty_like(xd)
    im = torch.empty_like(xd)
    _capi.huygens_f32(xd, yd, sd, k, L, re, im, xd.numel(), src.shape[0])
    torch.cuda.synchronize()
    return re.cpu().numpy(), im.cpu().numpy()


@pytest.mark.parametrize("P,S", [(1, 1), (5, 3), (4099, 1000), (1025, 4097), (3, 0)])
def test_bit_exact_small(torch_dev, P, S):
    rng = np.random.default_rng(P + S)
    src = np.stack([rng.uniform(-100, 100, S), rng.uniform(-100, 100, S), rng.uniform(0, 1, S) / max(S, 1),
                    rng.uniform(-math.pi, math.pi, S)], 1).astype(np.float32).reshape(S, 4)
    xo = rng.uniform(-300, 300, P).astype(np.float32)
    yo = rng.uniform(-300, 300, P).astype(np.float32)
    re, im = run(torch_dev, xo, yo, src, 2 * math.pi, 4000.0)
    ro, io = oracle.huygens(xo, yo, src, 2 * math.pi, 4000.0, threads=oracle.default_threads())
    assert_bit_exact(re, ro, "re P=%d S=%d" % (P, S))
    assert_bit_exact(im, io, "im P=%d S=%d" % (P, S))


@pytest.mark.slow
def test_diffraction_workload_sampled(torch_dev):
    """512 x 512 screen, 64 x 64 sources (lens + aberration): every sampled
    point bit-exact against the oracle."""
    from paper_cs_0406049_amd import workloads
    p = workloads.huygens_problem()
    re, im = run(torch_dev, p.xo, p.yo, p.src, p.k, p.L)
    idx = np.random.default_rng(0).choice(p.xo.size, 3000, replace=False)
    idx = np.concatenate([idx, [0, p.xo.size - 1, p.xo.size // 2 + 256]])
    ro, io = oracle.huygens(p.xo[idx], p.yo[idx], p.src, p.k, p.L, threads=oracle.default_threads())
    assert_bit_exact(re[idx], ro, "re (sample)")
    assert_bit_exact(im[idx], io, "im (sample)")
    inten = re.astype(np.float64) ** 2 + im.astype(np.float64) ** 2
    peak = int(np.argmax(inten))
    log("diffraction: peak intensity %.3g at (%.1f, %.1f), centre %.3g" % (
        inten[peak], p.xo[peak], p.yo[peak], inten[p.xo.size // 2 + 256]))
    # the lens focuses on the screen centre
    assert abs(p.xo[peak]) < 2.0 and abs(p.yo[peak]) < 2.0


def test_validation(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    x = torch.zeros(8, device="cuda")
    src = torch.zeros(16, device="cuda")
    out = torch.empty(8, device="cuda")
    out2 = torch.empty(8, device="cuda")
    with pytest.raises(_capi.SincosError):
        _capi.huygens_f32(x, x, src, 1.0, -1.0, out, out2)          # L <= 0
    with pytest.raises(_capi.SincosError):
        _capi.huygens_f32(x, x, src, 1.0, 1e18, out, out2)          # L >= 1e18
    with pytest.raises(_capi.SincosError):
        _capi.huygens_f32(x, x, src, 1.0, 10.0, out, out)           # re == im
    with pytest.raises(_capi.SincosError):
        _capi.huygens_f32(x, x, src[1:].data_ptr(), 1.0, 10.0, out, out2, 8, 3)  # src misaligned


@pytest.mark.parametrize("P,reps", [(1, 1), (4099, 3), (777, 0), (300, 17)])
def test_term_ceiling_is_the_sum_over_the_repeated_table(torch_dev, P, reps):
    """huygens_term_ceiling_f32 computes huygens_f32 over its 8 sources
    repeated reps times: bit-exact against the oracle on the tiled table."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, workloads
    p = workloads.huygens_problem(screen_side=64, aperture_side=8, seed=P + reps)
    rng = np.random.default_rng(P)
    idx = rng.choice(p.xo.size, min(P, p.xo.size), replace=False)
    xo = np.resize(p.xo[idx], P).astype(np.float32)
    yo = np.resize(p.yo[idx], P).astype(np.float32)
    src8 = np.ascontiguousarray(p.src[rng.choice(p.src.shape[0], 8, replace=False)])
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()  # noqa: E731
    xd, yd, sd = d(xo), d(yo), d(src8.reshape(-1))
    re = torch.full_like(xd, float("nan"))
    im = torch.full_like(xd, float("nan"))
    _capi.huygens_term_ceiling_f32(xd, yd, sd, reps, p.k, p.L, re, im)
    torch.cuda.synchronize()
    tiled = np.tile(src8, (reps, 1)) if reps else np.zeros((0, 4), np.float32)
    ro, io = oracle.huygens(xo, yo, tiled, p.k, p.L, threads=oracle.default_threads())
    assert_bit_exact(re.cpu().numpy(), ro, "ceiling re P=%d reps=%d" % (P, reps))
    assert_bit_exact(im.cpu().numpy(), io, "ceiling im P=%d reps=%d" % (P, reps))
    with pytest.raises(_capi.SincosError):
        _capi.huygens_term_ceiling_f32(xd, yd, sd, -1, p.k, p.L, re, im)


def _mixed(rng, P, S, big, every_src, every_pt):
    """Ordinary coordinates with every `every_src`-th source and every
    `every_pt`-th screen point moved to +-big."""
    src = np.stack([rng.uniform(-100, 100, S), rng.uniform(-100, 100, S), rng.uniform(0, 1, S) / S,
                    rng.uniform(-math.pi, math.pi, S)], 1).astype(np.float32)
    xo = rng.uniform(-300, 300, P).astype(np.float32)
    yo = rng.uniform(-300, 300, P).astype(np.float32)
    sgn = lambda n: np.where(rng.random(n) < 0.5, -1.0, 1.0)  # noqa: E731
    if every_src:
        j = np.arange(0, S, every_src)
        src[j, j % 2] = (sgn(j.size) * big).astype(np.float32)
    if every_pt:
        i = np.arange(0, P, every_pt)
        (xo if every_pt % 2 else yo)[i] = (sgn(i.size) * big).astype(np.float32)
    return xo, yo, src


@pytest.mark.parametrize("big,every_src,every_pt", [
    (2.0 ** 61, 7, 0),           # some groups take the IEEE reciprocal
    (2.0 ** 61, 0, 97),          # some waves take it for every group
    (2.0 ** 61, 5, 131),         # both
    (float(np.nextafter(np.float32(2.0 ** 60), np.float32(0))), 3, 89),  # just inside: rcp_rn
    (2.0 ** 60, 3, 89)])         # exactly 2^60: the IEEE reciprocal
def test_bit_exact_with_huge_coordinates(torch_dev, big, every_src, every_pt):
    """Coordinates at or above 2^60 in magnitude route a group (sources) or a
    whole wave (screen points) to the IEEE reciprocal; the results are the
    oracle's bits either way, next to the groups that take rcp_rn."""
    rng = np.random.default_rng(every_src * 1000 + every_pt)
    P, S = 1000, 203
    xo, yo, src = _mixed(rng, P, S, big, every_src, every_pt)
    re, im = run(torch_dev, xo, yo, src, 2 * math.pi, 4000.0)
    ro, io = oracle.huygens(xo, yo, src, 2 * math.pi, 4000.0, threads=oracle.default_threads())
    assert_bit_exact(re, ro, "re big=%g" % big)
    assert_bit_exact(im, io, "im big=%g" % big)


@pytest.mark.parametrize("L", [9.9e17, 2.0 ** -50, 1.0e-20])
def test_bit_exact_at_extreme_screen_distances(torch_dev, L):
    """L near the largest the call takes (1e18): rcp_rn with r (r + L) near
    2e36; L^2 < 2^-96: the general IEEE square root and the IEEE reciprocal
    (or the two divisions where r (r + L) is subnormal).  Coordinates scaled
    to L."""
    rng = np.random.default_rng(int(abs(math.log2(L))))
    P, S = 777, 131
    scale = np.float32(min(L, 1.0) * 0.01) if L < 1 else np.float32(1.0)
    src = np.stack([rng.uniform(-100, 100, S) * scale, rng.uniform(-100, 100, S) * scale,
                    rng.uniform(0, 1, S) / S, rng.uniform(-math.pi, math.pi, S)], 1).astype(np.float32)
    xo = (rng.uniform(-300, 300, P) * scale).astype(np.float32)
    yo = (rng.uniform(-300, 300, P) * scale).astype(np.float32)
    k = 2 * math.pi if L >= 1 else 2 * math.pi / float(scale)
    re, im = run(torch_dev, xo, yo, src, k, L)
    ro, io = oracle.huygens(xo, yo, src, k, L, threads=oracle.default_threads())
    assert_bit_exact(re, ro, "re L=%g" % L)
    assert_bit_exact(im, io, "im L=%g" % L)
