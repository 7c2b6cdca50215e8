"""The request server on the GPU: every result in the mix is the same bits
as the same request alone (plain call) and as the oracle; batches overlap."""
import numpy as np
import pytest

import oracle
from gpu_util import assert_bit_exact, device_view, lib_loaded, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    return torch


def _pool(torch, elems, seed):
    xh = np.random.default_rng(seed).uniform(-1e3, 1e3, elems).astype(np.float32)
    return xh, torch.from_numpy(xh).cuda()


@pytest.mark.parametrize("mode,stream_per_slot,split", [
    (0, False, 0),        # the default: each size class's batches in order on its stream
    (0, False, 4096),     # both classes present, on two streams
    (0, True, 4096),      # every batch on its slot's stream
    (1, True, 0)])        # one plain launch per request
def test_mix_equals_alone(torch_dev, mode, stream_per_slot, split):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, serve
    xh, pool = _pool(torch, 1 << 22, 1)
    rng = np.random.default_rng(2)
    sizes = np.floor(10 ** rng.uniform(0, 5.5, 300)).astype(np.int64)
    offs = rng.integers(0, pool.numel() - sizes.max() - 4, 300)
    offs[::5] += rng.integers(1, 4, offs[::5].size)   # some inputs off the 16-byte grid
    assert np.all(offs >= 0) and np.all(offs + sizes <= pool.numel())
    base = pool.data_ptr()
    with serve.Server(max_inflight=3, mode=mode, stream_per_slot=stream_per_slot,
                      split_elems=split) as srv:
        ids = [srv.submit(base + 4 * int(o), int(n), tag=j) for j, (o, n) in enumerate(zip(offs, sizes))]
        comps = []
        while len(comps) < len(ids):
            comps += srv.poll(256, 1.0)
        st = srv.stats()
        for c in comps:
            assert c.status == _capi.OK
            j = int(c.tag)
            n, o = int(sizes[j]), int(offs[j])
            s_alone = torch.empty(n, device="cuda")
            c_alone = torch.empty(n, device="cuda")
            _capi.sincos_f32(base + 4 * o, s_alone, c_alone, n)
            torch.cuda.synchronize()
            s_mix = device_view(torch, c.s, n).clone()
            c_mix = device_view(torch, c.c, n).clone()
            torch.cuda.synchronize()
            assert torch.equal(s_mix.view(torch.int32), s_alone.view(torch.int32)), j
            assert torch.equal(c_mix.view(torch.int32), c_alone.view(torch.int32)), j
            if j % 25 == 0:
                so, co = oracle.sincos(xh[o:o + n], 0, 0)
                assert_bit_exact(s_mix.cpu().numpy(), so, "served sin %d" % j)
                assert_bit_exact(c_mix.cpu().numpy(), co, "served cos %d" % j)
            srv.release(c.id)
        log("mode %d, stream per slot %d, split %d: %d requests in %d batches, inflight peak %d"
            % (mode, stream_per_slot, split, st["completed"], st["batches"], st["inflight_peak"]))
        assert srv.stats()["budget_in_use"] == 0


def test_replay_poisson_stream(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd import serve, workloads
    rs = workloads.request_stream(count=2000, seed=4, pool_elems=1 << 24)
    pool = torch.from_numpy(rs.pool).cuda()
    sizes = np.minimum(rs.sizes, 1 << 20)
    offs = np.minimum(rs.offsets, pool.numel() - sizes)
    offs -= offs % 64
    assert np.all(offs >= 0) and np.all(offs + sizes <= pool.numel())
    xs = [pool.data_ptr() + 4 * int(o) for o in offs]
    rate = 1e5                                   # requests per second
    arr = (np.cumsum(rs.unit_gaps) / rate * 1e9).astype(np.int64)
    with serve.Server(max_inflight=4, auto_release=True) as srv:
        comp = srv.replay(xs, sizes, arr)
        st = srv.stats()
    assert np.all(comp["status"] == 0)
    with serve.Server(auto_release=True) as srv:      # auto-released: no outputs to alias
        srv.submit(xs[0], int(sizes[0]))
        done = srv.poll(1, 5.0)
        assert done and done[0].status == 0
        with pytest.raises(ValueError):
            srv.outputs(done[0])
    summ = serve.latency_summary(comp)
    log("replay: %s, batches %d, inflight peak %d" % (summ, st["batches"], st["inflight_peak"]))
    assert st["batches"] < comp.size
    assert summ["p99_us"] > 0


def test_tight_budget_forces_waiting_and_keeps_results(torch_dev):
    """A budget of a few requests: admission waits for releases, batches stay
    small, every result is still the same as the request alone."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, serve
    xh, pool = _pool(torch, 1 << 20, 3)
    sizes = np.random.default_rng(4).integers(1000, 60000, 120)
    offs = np.random.default_rng(5).integers(0, pool.numel() - 60000, 120)
    assert np.all(offs + sizes <= pool.numel())
    base = pool.data_ptr()
    budget = 12 * 3 * 60000
    with serve.Server(budget_bytes=budget, max_inflight=2) as srv:
        comps = srv.replay([base + 4 * int(o) for o in offs], sizes, np.zeros(120, np.int64))
        st = srv.stats()
        assert st["budget_peak"] <= budget
        assert st["batches"] >= 120 * 1000 * 12 // budget
    assert np.all(comps["status"] == 0)
    # with auto_release off the replay released every request after storing it;
    # recompute a few alone and compare against a second, unconstrained run
    with serve.Server(max_inflight=4) as srv:
        for j in range(0, 120, 17):
            n, o = int(sizes[j]), int(offs[j])
            rid = srv.submit(base + 4 * o, n)
            c = None
            while c is None:
                got = srv.poll(4, 1.0)
                c = got[0] if got else None
            s_alone = torch.empty(n, device="cuda")
            c_alone = torch.empty(n, device="cuda")
            _capi.sincos_f32(base + 4 * o, s_alone, c_alone, n)
            torch.cuda.synchronize()
            assert torch.equal(device_view(torch, c.s, n).view(torch.int32), s_alone.view(torch.int32))
            assert torch.equal(device_view(torch, c.c, n).view(torch.int32), c_alone.view(torch.int32))
            srv.release(rid)


@pytest.mark.slow
def test_served_workload_full_sampled(torch_dev):
    """The served workload at full size: 10,000 requests of log-uniform size
    in [1e3, 1e7] (about 1.1e10 elements), the 8 GiB budget and four batches
    in flight, all submitted at once.  Every request completes; each result,
    read before its release, agrees bit for bit with the oracle on sampled
    elements (the first 8, the last 8 and 48 random positions)."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, serve, workloads
    rs = workloads.request_stream()
    pool = torch.from_numpy(rs.pool).cuda()
    assert int((rs.offsets + rs.sizes).max()) <= pool.numel()
    base = pool.data_ptr()
    rng = np.random.default_rng(9)
    xs, ss, cs = [], [], []
    with serve.Server(max_inflight=4) as srv:
        for j, (o, n) in enumerate(zip(rs.offsets, rs.sizes)):
            srv.submit(base + 4 * int(o), int(n), tag=j)
        left = rs.sizes.size
        while left:
            got = srv.poll(256, 5.0)
            assert got, "no completion within 5 s"
            for c in got:
                assert c.status == _capi.OK
                j = int(c.tag)
                n, o = int(rs.sizes[j]), int(rs.offsets[j])
                assert c.n == n
                idx = np.unique(np.concatenate([np.arange(8), np.arange(n - 8, n),
                                                rng.integers(0, n, 48)]))
                ti = torch.from_numpy(idx).cuda()
                ss.append(device_view(torch, c.s, n).index_select(0, ti).cpu().numpy())
                cs.append(device_view(torch, c.c, n).index_select(0, ti).cpu().numpy())
                xs.append(rs.pool[o + idx])
                srv.release(c.id)
            left -= len(got)
        st = srv.stats()
    assert st["completed"] == rs.sizes.size and st["failed"] == 0
    assert st["budget_in_use"] == 0 and st["budget_peak"] <= 8 << 30
    x = np.concatenate(xs)
    so, co = oracle.sincos(x, 0, 0, threads=oracle.default_threads())
    assert_bit_exact(np.concatenate(ss), so, "served full workload sin", x)
    assert_bit_exact(np.concatenate(cs), co, "served full workload cos", x)
    log("served full workload: %d requests, %d batches, inflight peak %d, %d sampled outputs" % (
        st["completed"], st["batches"], st["inflight_peak"], x.size))


def test_submit_waits_for_the_producing_stream_and_keeps_the_input(torch_dev):
    """Inputs still being written on the current stream (host-to-device copies
    queued behind a few milliseconds of matrix products) are submitted and
    dropped at once.  The batches wait for the copies on the device, and the
    server holds each tensor until its completion is polled, so the allocator
    cannot hand its memory to the zero-filled tensors made right after: every
    result is the oracle's bits."""
    torch = torch_dev
    from paper_cs_0406049_amd import serve
    rng = np.random.default_rng(21)
    sizes = [1000, 65536 + 3, 1 << 20]
    hosts = [rng.uniform(-1e3, 1e3, n).astype(np.float32) for n in sizes]
    pinned = [torch.from_numpy(h).pin_memory() for h in hosts]
    a = torch.randn(4096, 4096, device="cuda")
    b = torch.randn(4096, 4096, device="cuda") / 64.0
    with serve.Server(max_inflight=2) as srv:
        for j, h in enumerate(hosts):
            x = torch.full((h.size,), float("nan"), device="cuda")
            torch.cuda.synchronize()
            for _ in range(4):
                a = torch.mm(a, b)          # keeps the current stream busy
            x.copy_(pinned[j], non_blocking=True)
            srv.submit(x, tag=j)
            del x
            junk = torch.zeros(h.size, device="cuda")
            del junk
        comps = []
        while len(comps) < len(sizes):
            comps += srv.poll(16, 5.0)
        assert not srv._inputs
        for c in comps:
            j = int(c.tag)
            s, co = serve.Server.outputs(c)
            so, cw = oracle.sincos(hosts[j], 0, 0)
            assert_bit_exact(s.cpu().numpy(), so, "served sin %d" % j)
            assert_bit_exact(co.cpu().numpy(), cw, "served cos %d" % j)
            srv.release(c.id)
    torch.cuda.synchronize()
    log("submit_on: %d fresh inputs served bit-exact" % len(sizes))
