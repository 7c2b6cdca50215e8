"""The library under HIP graph capture and from several host threads."""
import threading

import numpy as np
import pytest

import oracle
from gpu_util import assert_bit_exact, lib_loaded

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    return torch


def test_plain_and_backward_in_a_captured_graph(torch_dev):
    """sincos_f32 and sincos_f32_backward are single kernel launches with no
    host work, so they can be captured; each replay (with eager work and new
    inputs in between) matches the oracle on that replay's inputs."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    n = 1_000_003
    x = torch.empty(n, device="cuda")
    gs = torch.empty(n, device="cuda")
    gc = torch.empty(n, device="cuda")
    s, c, gx = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    x.uniform_(-100, 100)
    gs.normal_()
    gc.normal_()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):        # warm-up outside capture
        _capi.sincos_f32(x, s, c, n)
        _capi.sincos_f32_backward(s, c, gs, gc, gx, n)
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        _capi.sincos_f32(x, s, c, n)
        _capi.sincos_f32_backward(s, c, gs, gc, gx, n)
    for rep in range(3):
        rng = np.random.default_rng(rep)
        xh = rng.uniform(-1e3, 1e3, n).astype(np.float32)
        gsh = rng.standard_normal(n).astype(np.float32)
        gch = rng.standard_normal(n).astype(np.float32)
        x.copy_(torch.from_numpy(xh))
        gs.copy_(torch.from_numpy(gsh))
        gc.copy_(torch.from_numpy(gch))
        _ = (torch.randn(1 << 18, device="cuda") * 2).sum()       # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        so, co = oracle.sincos(xh, 0, 0, threads=oracle.default_threads())
        assert_bit_exact(s.cpu().numpy(), so, "replay %d sin" % rep)
        assert_bit_exact(c.cpu().numpy(), co, "replay %d cos" % rep)
        assert_bit_exact(gx.cpu().numpy(), oracle.sincos_backward(so, co, gsh, gch), "replay %d gx" % rep)


def test_fit_step_in_a_captured_graph(torch_dev):
    """One least-squares fit step (fused residual and loss, adjoint with its
    reduction) captured as a graph: no allocation or synchronization happens
    inside the library calls, and the kernels sum in a fixed order, so every
    replay gives the same bits as the eager call on the same inputs."""
    torch = torch_dev
    from paper_cs_0406049_amd import workloads
    from paper_cs_0406049_amd.autograd import sinusoid_loss_and_grads
    p = workloads.sinusoid_problem(N=300_000, K=64)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).cuda()  # noqa: E731
    t, yobs, A, w, phi = d(p.t), d(p.y_obs), d(p.A), d(p.w), d(p.phi)
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):        # warm-up outside capture
        sinusoid_loss_and_grads(t, yobs, A, w, phi)
    torch.cuda.current_stream().wait_stream(st)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=st):
        out = sinusoid_loss_and_grads(t, yobs, A, w, phi)
    for rep in range(3):
        rng = np.random.default_rng(100 + rep)
        A.copy_(d(p.A + 0.01 * rng.standard_normal(p.A.size)))
        phi.copy_(d(p.phi + 0.01 * rng.standard_normal(p.phi.size)))
        _ = (torch.randn(1 << 18, device="cuda") * 2).sum()       # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [o.detach().clone() for o in out]
        want = sinusoid_loss_and_grads(t, yobs, A, w, phi)
        torch.cuda.synchronize()
        for k, (a, b) in enumerate(zip(got, want)):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32)), (rep, k)


def test_ragged_from_many_threads_on_their_own_streams(torch_dev):
    """Several host threads enqueue one-shot ragged batches (sharing the
    library's staging ring) on their own streams at the same time."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    threads, rounds = 6, 12
    errors = []
    results = {}

    def worker(t):
        try:
            rng = np.random.default_rng(100 + t)
            st = torch.cuda.Stream()
            lens = rng.integers(1, 20000, 40)
            xs = [rng.uniform(-1e3, 1e3, int(m)).astype(np.float32) for m in lens]
            with torch.cuda.stream(st):
                xd = [torch.from_numpy(a).cuda() for a in xs]
                outs = [(torch.empty_like(a), torch.empty_like(a)) for a in xd]
                for _ in range(rounds):
                    _capi.sincos_f32_ragged([(a, s_, c_) for a, (s_, c_) in zip(xd, outs)], lens,
                                            stream=st)
            st.synchronize()
            results[t] = (xs, [(s_.cpu().numpy(), c_.cpu().numpy()) for s_, c_ in outs])
        except Exception as e:  # reported below
            errors.append(repr(e))

    ths = [threading.Thread(target=worker, args=(t,)) for t in range(threads)]
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    assert not errors, errors
    for t, (xs, outs) in results.items():
        for a, (sg, cg) in zip(xs, outs):
            so, co = oracle.sincos(a, 0, 0)
            assert_bit_exact(sg, so, "thread %d sin" % t)
            assert_bit_exact(cg, co, "thread %d cos" % t)
