"""The memory-traffic probes do what sincos.h says: every copy schedule gives
s = c = x bit for bit over whole tiles and ragged last tiles, in every cache
policy and LDS reservation it is measured with; the write probes fill s and c
(WRITE1 leaves c alone) without touching anything past n; the read probe
writes nothing for ordinary inputs.  And the plain kernel gives the oracle's
bits with any LDS reservation."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_bit_exact, lib_loaded

pytestmark = pytest.mark.gpu

GUARD = 64


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    return torch


def _buffers(torch, n):
    """x, s, c views of n floats followed by GUARD canary floats each."""
    rng = np.random.default_rng(n)
    xh = rng.uniform(-50, 50, n).astype(np.float32)
    bufs = [torch.full((n + GUARD,), float("nan"), device="cuda") for _ in range(3)]
    bufs[0][:n] = torch.from_numpy(xh).cuda()
    return xh, bufs


def _guards_intact(torch, bufs, n):
    for b in bufs:
        assert torch.isnan(b[n:]).all(), "a probe wrote past n"


@pytest.mark.parametrize("n", [4, 256, 1024 + 4, 64 * 1024 * 3 + 512 + 12, 1 << 22])
def test_copy_schedules_copy(torch_dev, n):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi as P
    xh, (x, s, c) = _buffers(torch, n)
    cases = [(P.PROBE_COPY, (64, 1, 0, -1), -1), (P.PROBE_COPY, (64, 1, 0, 7168), -1),
             (P.PROBE_COPY, (256, 4, 0, -1), 18), (P.PROBE_COPY, (64, 8, 3, -1), 2),
             (P.PROBE_COPY, (128, 2, 0, 0), 0), (P.PROBE_COPY, (64, 1, 0, -1), 1),
             (P.PROBE_COPY, (64, 1, 0, -1), 16), (P.PROBE_COPY, (64, 1, 0, -1), 17),
             (P.PROBE_COPY_BATCH, (64, 2, 0, -1), -1), (P.PROBE_COPY_BATCH, (256, 8, 5, -1), -1),
             (P.PROBE_COPY_SPLIT, (64, 1, 0, -1), -1), (P.PROBE_COPY_SPLIT, (64, 1, 7, -1), -1),
             (P.PROBE_COPY_LDS, (64, 1, 0, -1), -1), (P.PROBE_COPY_LDS, (64, 1, 3, 16384), -1),
             (P.PROBE_COPY_XCD, (64, 1, 0, -1), -1), (P.PROBE_COPY_XCD, (256, 1, 0, 8192), -1),
             (P.PROBE_COPY_XCD, (64, 1, 1, -1), -1), (P.PROBE_COPY_XCD, (64, 1, 2, -1), -1),
             (P.PROBE_COPY_XCD, (64, 1, 7, 8192), -1)]
    for probe, shape, policy in cases:
        s[:n].fill_(float("nan"))
        c[:n].fill_(float("nan"))
        P.sincos_stream_probe_f32(probe, x[:n], s[:n], c[:n], n, launch=shape, policy=policy)
        torch.cuda.synchronize()
        what = "%s %s policy %d n=%d" % (P.PROBE_NAMES[probe], shape, policy, n)
        assert_bit_exact(s[:n].cpu().numpy(), xh, what + " s")
        assert_bit_exact(c[:n].cpu().numpy(), xh, what + " c")
        _guards_intact(torch, (x, s, c), n)


@pytest.mark.parametrize("n", [4, 1024 + 4, 1 << 20])
def test_write_and_read_probes(torch_dev, n):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi as P
    xh, (x, s, c) = _buffers(torch, n)
    for shape, policy in (((64, 1, 0, -1), -1), ((64, 1, 0, 16384), 18), ((256, 2, 0, -1), 0)):
        s[:n].fill_(float("nan"))
        c[:n].fill_(float("nan"))
        P.sincos_stream_probe_f32(P.PROBE_WRITE, None, s[:n], c[:n], n, launch=shape,
                                  policy=policy)
        torch.cuda.synchronize()
        sv, cv = s[:n].cpu().numpy(), c[:n].cpu().numpy()
        assert np.array_equal(sv.view(np.uint32), cv.view(np.uint32))
        assert not np.isnan(sv).all(), "write probe left s unwritten"
        _guards_intact(torch, (x, s, c), n)
        s[:n].fill_(float("nan"))
        c[:n].fill_(float("nan"))
        P.sincos_stream_probe_f32(P.PROBE_WRITE1, None, s[:n], None, n, launch=shape,
                                  policy=policy)
        torch.cuda.synchronize()
        assert np.array_equal(s[:n].cpu().numpy().view(np.uint32), sv.view(np.uint32))
        assert torch.isnan(c).all(), "one-stream write probe touched c"
        _guards_intact(torch, (x, s, c), n)
    for shape, policy in (((1024, 1, 0, -1), -1), ((64, 4, 0, 8192), 0), ((256, 1, 0, -1), 16)):
        s.fill_(float("nan"))
        P.sincos_stream_probe_f32(P.PROBE_READ, x[:n], s[:1], None, n, launch=shape, policy=policy)
        torch.cuda.synchronize()
        assert torch.isnan(s).all(), "read probe wrote for ordinary input"
    assert_bit_exact(x[:n].cpu().numpy(), xh, "probe input unchanged")


def test_plain_kernel_with_lds_reservations(torch_dev):
    """The LDS reservation changes only residency: same bits as the oracle."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    n = (1 << 21) + 7
    xh, (x, s, c) = _buffers(torch, n)
    so, co = oracle.sincos(xh, 0, 0, threads=oracle.default_threads())
    for lds in (-1, 0, 512, 7168, 16384, 65536):
        s.fill_(float("nan"))
        c.fill_(float("nan"))
        _capi.sincos_f32_ex(x[:n], s[:n], c[:n], n, launch=(64, 1, 0, lds))
        torch.cuda.synchronize()
        assert_bit_exact(s[:n].cpu().numpy(), so, "lds %d sin" % lds, xh)
        assert_bit_exact(c[:n].cpu().numpy(), co, "lds %d cos" % lds, xh)
        _guards_intact(torch, (x, s, c), n)
