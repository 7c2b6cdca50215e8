"""Arrays past 2^31 elements (8 GiB in, 16 GiB out): 64-bit indexing, one
workgroup per tile (the default grid: 2^23 workgroups here) and, with a grid
of 2^20 workgroups, the grid-stride loop, and the per-tile buffer ranges,
checked against the oracle on sampled outputs (the oracle computes each one
alone): random indices, both ends, and the neighbourhoods of 2^31 and of
every multiple of 2^28 elements (where a 2^20-workgroup grid wraps at 64
float4 per workgroup)."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_bit_exact, lib_loaded, log

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

N_BIG = (1 << 31) + 3          # a ragged tail of 3 past the last float4


@pytest.fixture(scope="module")
def big(request):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    free, _ = torch.cuda.mem_get_info()
    if free < 40 << 30:
        pytest.skip("needs about 40 GiB of free device memory")
    g = torch.Generator(device="cuda")
    g.manual_seed(31)
    x = torch.empty(N_BIG, device="cuda").uniform_(-1e4, 1e4, generator=g)
    yield torch, x
    del x
    torch.cuda.empty_cache()


def sample_indices(n, seed):
    rng = np.random.default_rng(seed)
    idx = [rng.integers(0, n, 100_000), np.arange(0, 2000), np.arange(n - 2000, n)]
    for k in range(1, n // (1 << 28) + 1):
        b = k * (1 << 28)
        idx.append(np.arange(max(0, b - 70), min(n, b + 70)))
    b = 1 << 31
    idx.append(np.arange(b - 70, min(n, b + 70)))
    return np.unique(np.concatenate(idx)).astype(np.int64)


def check_sampled(torch, x, s, c, n, arith, what):
    idx = sample_indices(n, 7 + arith)
    ti = torch.from_numpy(idx).cuda()
    xh = x.index_select(0, ti).cpu().numpy()
    so, co = oracle.sincos(xh, arith, 0, threads=oracle.default_threads())
    assert_bit_exact(s.index_select(0, ti).cpu().numpy(), so, what + " sin", xh)
    assert_bit_exact(c.index_select(0, ti).cpu().numpy(), co, what + " cos", xh)
    return idx.size


@pytest.mark.parametrize("arith,grid", [(0, 0), (1, 0), (0, 1 << 20)])
def test_plain_past_2_31(big, arith, grid):
    torch, x = big
    from paper_cs_0406049_amd import _capi
    s = torch.empty_like(x)
    c = torch.empty_like(x)
    s.fill_(float("nan"))
    c.fill_(float("nan"))
    _capi.sincos_f32_ex(x, s, c, N_BIG, arith, 0, launch=(64, 1, grid, 0) if grid else None)
    torch.cuda.synchronize()
    what = "plain n=2^31+3 arith %d grid %d" % (arith, grid)
    k = check_sampled(torch, x, s, c, N_BIG, arith, what)
    log("%s: %d sampled outputs bit-exact" % (what, k))
    del s, c


def test_ragged_segment_past_2_31(big):
    """One ragged call: a segment longer than 2^31 elements next to small ones."""
    torch, x = big
    from paper_cs_0406049_amd import _capi
    small = x[:1000].clone()
    s = torch.empty_like(x)
    c = torch.empty_like(x)
    s2 = torch.empty_like(small)
    c2 = torch.empty_like(small)
    _capi.sincos_f32_ragged([(small, s2, c2), (x, s, c)], [1000, N_BIG])
    torch.cuda.synchronize()
    check_sampled(torch, x, s, c, N_BIG, 0, "ragged big segment")
    so, co = oracle.sincos(small.cpu().numpy(), 0, 0)
    assert_bit_exact(s2.cpu().numpy(), so, "ragged small segment sin")
    assert_bit_exact(c2.cpu().numpy(), co, "ragged small segment cos")
    del s, c


def test_interleaved_past_2_31(big):
    torch, x = big
    from paper_cs_0406049_amd import _capi
    out = torch.empty(2 * N_BIG, device="cuda")
    _capi.sincos_f32_interleaved(x, out, N_BIG, 0)
    torch.cuda.synchronize()
    idx = sample_indices(N_BIG, 11)
    ti = torch.from_numpy(idx).cuda()
    xh = x.index_select(0, ti).cpu().numpy()
    so, co = oracle.sincos(xh, 0, 0, threads=oracle.default_threads())
    assert_bit_exact(out.index_select(0, 2 * ti).cpu().numpy(), co, "interleaved cos", xh)
    assert_bit_exact(out.index_select(0, 2 * ti + 1).cpu().numpy(), so, "interleaved sin", xh)
    del out
