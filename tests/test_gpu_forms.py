"""Ragged, adjoint and sinusoid forms on the GPU against the CPU oracle."""
import math

import numpy as np
import pytest

import oracle
from gpu_util import assert_bit_exact, lib_loaded, log

pytestmark = pytest.mark.gpu

U = 2.0 ** -24


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    lib_loaded()
    return torch


# ---------------------------------------------------------------------------
# Ragged form


def _segments(torch, lens, seed, lo=-100 * math.pi, hi=100 * math.pi):
    rng = np.random.default_rng(seed)
    xs_h = [rng.uniform(lo, hi, int(n)).astype(np.float32) for n in lens]
    segs = []
    for xh in xs_h:
        x = torch.from_numpy(xh).cuda() if xh.size else torch.empty(0, device="cuda")
        segs.append((x, torch.empty_like(x), torch.empty_like(x)))
    return xs_h, segs


def _check_segments(xs_h, segs, what, arith=0):
    for j, (xh, (_, s, c)) in enumerate(zip(xs_h, segs)):
        if xh.size == 0:
            continue
        so, co = oracle.sincos(xh, arith, 0)
        assert_bit_exact(s.cpu().numpy(), so, "%s seg %d sin" % (what, j), xh)
        assert_bit_exact(c.cpu().numpy(), co, "%s seg %d cos" % (what, j), xh)


@pytest.mark.parametrize("launch", [None, (64, 1, 1), (256, 4, 0), (512, 2, 5), (1024, 8, 0),
                                    (128, 4, 10000)])
def test_ragged_mixed_lengths(torch_dev, launch):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    lens = [0, 1, 2, 3, 4, 5, 15, 16, 17, 100, 1023, 1024, 4097, 65535, 100000, 0, 7, 300000]
    xs_h, segs = _segments(torch, lens, 1)
    _capi.sincos_f32_ragged(segs, lens, launch=launch)
    torch.cuda.synchronize()
    _check_segments(xs_h, segs, "ragged %r" % (launch,))


@pytest.mark.parametrize("nonempty,empty", [(1, 0), (63, 0), (64, 0), (64, 9), (65, 0), (200, 3)])
@pytest.mark.parametrize("arith,method", [(0, 0), (1, 1)])
def test_ragged_inline_and_staged_tables(torch_dev, nonempty, empty, arith, method):
    """Up to 64 non-empty segments the table travels in the kernel arguments;
    beyond, it is staged through device memory.  Both give the oracle's
    bits, at and around the boundary, with empty segments interleaved."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    rng = np.random.default_rng(nonempty * 31 + empty)
    lens = [int(v) for v in rng.integers(1, 20000, nonempty)]
    for k in range(empty):
        lens.insert(int(rng.integers(0, len(lens) + 1)), 0)
    xs_h, segs = _segments(torch, lens, nonempty + empty)
    _capi.sincos_f32_ragged(segs, lens, arith=arith, method=method)
    torch.cuda.synchronize()
    for j, (xh, (_, s, c)) in enumerate(zip(xs_h, segs)):
        if xh.size == 0:
            continue
        so, co = oracle.sincos(xh, arith, method)
        assert_bit_exact(s.cpu().numpy(), so, "ragged %d+%d seg %d sin" % (nonempty, empty, j), xh)
        assert_bit_exact(c.cpu().numpy(), co, "ragged %d+%d seg %d cos" % (nonempty, empty, j), xh)


def test_tuned_default_shapes_apply_and_keep_bits(torch_dev):
    """Shapes installed with sincos_set_tuning are used by calls that pass
    none (a ragged plan reports them) and leave every output bit unchanged."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    lens = [0, 1, 5, 17, 1023, 4097, 100000, 3]
    try:
        _capi.set_tuning({"plain": (512, 4, 7), "ragged": (128, 2, 9)})
        xs_h, segs = _segments(torch, lens, 11)
        _capi.sincos_f32_ragged(segs, lens)
        torch.cuda.synchronize()
        _check_segments(xs_h, segs, "ragged, tuned default")
        plan = _capi.RaggedPlan(segs, lens)
        i = plan.info()
        assert (i["block"], i["unroll"], i["grid"]) == (128, 2, 9)
        plan.destroy()
        x = torch.from_numpy(xs_h[6]).cuda()
        s, c = torch.empty_like(x), torch.empty_like(x)
        _capi.sincos_f32(x, s, c)
        torch.cuda.synchronize()
        so, co = oracle.sincos(xs_h[6], 0, 0)
        assert_bit_exact(s.cpu().numpy(), so, "plain, tuned default sin", xs_h[6])
        assert_bit_exact(c.cpu().numpy(), co, "plain, tuned default cos", xs_h[6])
    finally:
        _capi.set_tuning(None)


@pytest.mark.parametrize("arith", [0, 1])
def test_ragged_equals_per_array_plain(torch_dev, arith):
    """The ragged launch gives, per element, the same bits as one plain launch
    per array (the arithmetic is unchanged)."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, workloads
    lens = workloads.ragged_lengths(200, seed=11)
    xs_h, segs = _segments(torch, lens, 2)
    _capi.sincos_f32_ragged(segs, lens, arith=arith)
    for x, s, c in segs:
        s2, c2 = torch.empty_like(x), torch.empty_like(x)
        _capi.sincos_f32_ex(x, s2, c2, x.numel(), arith, 0)
        torch.cuda.synchronize()
        assert torch.equal(s.view(torch.int32), s2.view(torch.int32))
        assert torch.equal(c.view(torch.int32), c2.view(torch.int32))


def test_ragged_packed_buffer_odd_offsets(torch_dev):
    """Segments packed into shared buffers at arbitrary 4-byte offsets (mixed
    16-byte phases, so some segments take the scalar path), shared inputs, an
    in-place segment, and canaries between outputs."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    rng = np.random.default_rng(3)
    lens = [int(v) for v in rng.integers(1, 5000, 40)] + [3, 1, 70001]
    total = sum(lens) + 8 * len(lens) + 64
    X = torch.from_numpy(rng.uniform(-1e3, 1e3, total).astype(np.float32)).cuda()
    canary = np.uint32(0x7FC0BEEF)
    S = torch.from_numpy(np.full(total, canary, np.uint32).view(np.float32)).cuda()
    C = S.clone()
    segs, spans = [], []
    pos_x, pos_s, pos_c = 1, 2, 3
    for j, n in enumerate(lens):
        if j % 7 == 3 and j > 0:   # share the previous segment's input
            xo = spans[-1][0] if lens[j - 1] >= n else pos_x
        else:
            xo = pos_x
        segs.append((X[xo:xo + n], S[pos_s:pos_s + n], C[pos_c:pos_c + n]))
        spans.append((xo, pos_s, pos_c, n))
        pos_x += n + int(rng.integers(0, 5))
        pos_s += n + 1 + int(rng.integers(0, 5))
        pos_c += n + 1 + int(rng.integers(0, 5))
    Xh = X.cpu().numpy()
    ptr = lambda t: t.data_ptr()  # noqa: E731
    _capi.sincos_f32_ragged([(ptr(a), ptr(b), ptr(c)) for a, b, c in segs], lens)
    torch.cuda.synchronize()
    Sh = S.cpu().numpy()
    Ch = C.cpu().numpy()
    written = np.zeros(total, bool)
    for (xo, so_, co_, n) in spans:
        so, co = oracle.sincos(Xh[xo:xo + n], 0, 0)
        assert_bit_exact(Sh[so_:so_ + n], so, "packed sin")
        assert_bit_exact(Ch[co_:co_ + n], co, "packed cos")
        written[so_:so_ + n] = True
    assert np.all(Sh.view(np.uint32)[~written] == canary)
    # in-place segment
    xh = rng.uniform(-10, 10, 1001).astype(np.float32)
    x = torch.from_numpy(xh).cuda()
    c = torch.empty_like(x)
    _capi.sincos_f32_ragged([(x, x, c)], [x.numel()])
    torch.cuda.synchronize()
    so, co = oracle.sincos(xh, 0, 0)
    assert_bit_exact(x.cpu().numpy(), so, "in-place sin")
    assert_bit_exact(c.cpu().numpy(), co, "in-place cos")


def test_ragged_plan_and_graph_replays(torch_dev):
    """A plan's kernel and its graph replayed several times, with eager work
    and new input values between replays: every replay matches the oracle on
    the inputs current at that replay."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, workloads
    lens = workloads.ragged_lengths(300, seed=5)
    xs_h, segs = _segments(torch, lens, 4)
    plan = _capi.RaggedPlan(segs, lens)
    info = plan.info()
    assert info["elements"] == int(sum(lens))
    for rep in range(4):
        rng = np.random.default_rng(100 + rep)
        for j, (x, s, c) in enumerate(segs):
            xs_h[j] = rng.uniform(-1e3, 1e3, x.numel()).astype(np.float32)
            x.copy_(torch.from_numpy(xs_h[j]))
            s.fill_(float("nan"))
            c.fill_(float("nan"))
        _ = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work
        if rep % 2 == 0:
            plan.graph_launch()
        else:
            plan.launch()
        torch.cuda.synchronize()
        _check_segments(xs_h, segs, "replay %d" % rep)
    plan.destroy()


def test_ragged_refuses_capture(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    x = torch.zeros(16, device="cuda")
    s, c = torch.empty_like(x), torch.empty_like(x)
    st = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(_capi.SincosError, match="captured"):
        with torch.cuda.graph(g, stream=st):
            _capi.sincos_f32_ragged([(x, s, c)], [16])


@pytest.mark.slow
def test_ragged_batch_workload_full(torch_dev):
    """4096 arrays, lengths log-uniform in [100, 1e6], angles U[-100 pi,
    100 pi): one graph launch of the plan, every element against the oracle."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, workloads
    lens, xs_h = workloads.ragged_batch()
    segs = []
    for xh in xs_h:
        x = torch.from_numpy(xh).cuda()
        segs.append((x, torch.empty_like(x), torch.empty_like(x)))
    plan = _capi.RaggedPlan(segs, lens)
    plan.graph_launch()
    torch.cuda.synchronize()
    flat_x = np.concatenate(xs_h)
    so, co = oracle.sincos(flat_x, 0, 0, threads=oracle.default_threads())
    sg = torch.cat([s for _, s, _ in segs]).cpu().numpy()
    cg = torch.cat([c for _, _, c in segs]).cpu().numpy()
    assert_bit_exact(sg, so, "ragged workload sin", flat_x)
    assert_bit_exact(cg, co, "ragged workload cos", flat_x)
    log("ragged workload: %d segments, %d elements bit-exact" % (len(lens), flat_x.size))
    plan.destroy()


# ---------------------------------------------------------------------------
# Adjoint of the pair


@pytest.mark.parametrize("present", ["both", "gs", "gc", "none"])
@pytest.mark.parametrize("offset,gx_offset", [(0, 0), (1, 1), (3, 3), (0, 2)])
def test_pair_backward_bit_exact(torch_dev, present, offset, gx_offset):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    rng = np.random.default_rng(7)
    for n in (1, 5, 1000, 1 << 20):
        xh = rng.uniform(-10, 10, n).astype(np.float32)
        sh, ch = oracle.sincos(xh, 0, 0)
        gsh = rng.standard_normal(n).astype(np.float32)
        gch = rng.standard_normal(n).astype(np.float32)

        def dev(a, off=offset):
            buf = torch.zeros(n + off, device="cuda")
            buf[off:] = torch.from_numpy(a).cuda()
            return buf[off:]
        s, c = dev(sh), dev(ch)
        gs = dev(gsh) if present in ("both", "gs") else None
        gc = dev(gch) if present in ("both", "gc") else None
        gx = dev(np.zeros(n, np.float32), gx_offset)
        _capi.sincos_f32_backward(s, c, gs, gc, gx, n)
        torch.cuda.synchronize()
        want = oracle.sincos_backward(sh, ch, gsh if gs is not None else None,
                                      gch if gc is not None else None)
        assert_bit_exact(gx.cpu().numpy(), want, "backward %s n=%d" % (present, n))


def test_pair_backward_in_place_and_autograd(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    from paper_cs_0406049_amd.autograd import sincos
    rng = np.random.default_rng(8)
    xh = rng.uniform(-20, 20, 100003).astype(np.float32)
    gsh = rng.standard_normal(xh.size).astype(np.float32)
    gch = rng.standard_normal(xh.size).astype(np.float32)
    sh, ch = oracle.sincos(xh, 0, 0)
    want = oracle.sincos_backward(sh, ch, gsh, gch)
    # in place: gx overwrites gs
    s, c = torch.from_numpy(sh).cuda(), torch.from_numpy(ch).cuda()
    gs, gc = torch.from_numpy(gsh).cuda(), torch.from_numpy(gch).cuda()
    _capi.sincos_f32_backward(s, c, gs, gc, gs, xh.size)
    torch.cuda.synchronize()
    assert_bit_exact(gs.cpu().numpy(), want, "in-place backward")
    # through torch.autograd
    x = torch.from_numpy(xh).cuda().requires_grad_(True)
    so, co = sincos(x)
    (so * torch.from_numpy(gsh).cuda() + co * torch.from_numpy(gch).cuda()).sum().backward()
    assert_bit_exact(so.detach().cpu().numpy(), sh, "autograd forward")
    assert_bit_exact(x.grad.cpu().numpy(), want, "autograd backward")


# ---------------------------------------------------------------------------
# Sinusoid model


def _sinusoid_small(N, K, seed):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0, 1000, N).astype(np.float32)
    A = rng.standard_normal(K).astype(np.float32)
    w = rng.uniform(0.1, 10, K).astype(np.float32)
    phi = rng.uniform(-math.pi, math.pi, K).astype(np.float32)
    return t, A, w, phi


ADJ_CHUNK = 128   # samples per wave in the adjoint kernel
ADJ_WAVES = 16    # waves per workgroup, summed in a pairwise tree


def _adjoint_bound(N, abs_sum):
    """Rounding bound of the kernel's binary32 sums against exact sums:
    per-wave recursive fma sums over at most ADJ_CHUNK samples, a 4-level
    pairwise tree over the workgroup's waves, a strided per-thread pass over
    the workgroup partials (at most ceil(parts/256) terms) and an 8-level tree,
    plus the rounding of g*t and of the final A_k product."""
    chunks = max(1, -(-N // ADJ_CHUNK))
    parts = -(-chunks // ADJ_WAVES)
    depth = min(N, ADJ_CHUNK) + (ADJ_WAVES.bit_length() - 1) + -(-parts // 256) + 8 + 3
    return depth * U * abs_sum * 1.001


@pytest.mark.parametrize("N,K", [(1, 1), (1000, 3), (4099, 64), (20000, 65), (5000, 130),
                                 (300000, 64)])
def test_sinusoid_forward_bit_exact_and_adjoint_bound(torch_dev, N, K):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    t, A, w, phi = _sinusoid_small(N, K, N + K)
    d = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    td, Ad, wd, pd = d(t), d(A), d(w), d(phi)
    y = torch.empty_like(td)
    _capi.sinusoid_f32_forward(td, Ad, wd, pd, y)
    torch.cuda.synchronize()
    yo = oracle.sinusoid_forward(t, A, w, phi, threads=oracle.default_threads())
    assert_bit_exact(y.cpu().numpy(), yo, "sinusoid forward N=%d K=%d" % (N, K))
    t2 = d(t)                              # in place: y over t
    _capi.sinusoid_f32_forward(t2, Ad, wd, pd, t2)
    torch.cuda.synchronize()
    assert_bit_exact(t2.cpu().numpy(), yo, "sinusoid forward in place N=%d K=%d" % (N, K))
    g = np.random.default_rng(1).standard_normal(N).astype(np.float32)
    gA, gw, gp = (torch.empty_like(Ad) for _ in range(3))
    nb = _capi.sinusoid_f32_backward_workspace_bytes(N, K)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    _capi.sinusoid_f32_backward(td, d(g), Ad, wd, pd, gA, gw, gp, ws)
    torch.cuda.synchronize()
    ref = oracle.sinusoid_adjoint(t, g, A, w, phi)
    for key, got, absk in (("gA", gA, "abs_A"), ("gw", gw, "abs_w"), ("gphi", gp, "abs_phi")):
        err = np.abs(got.cpu().numpy().astype(np.float64) - ref[key])
        bound = _adjoint_bound(N, ref[absk]) + np.abs(ref[key]) * U
        assert np.all(err <= bound), (key, (err / np.maximum(bound, 1e-300)).max())


@pytest.mark.parametrize("N,K", [(1, 1), (1000, 3), (4099, 64), (300000, 64), (2049, 0)])
def test_sinusoid_residual_and_loss(torch_dev, N, K):
    """r = y - y_obs bit-exact (y as the oracle's forward), the loss within the
    rounding bound of its fixed-order binary32 sums; in place over y_obs too."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    t, A, w, phi = _sinusoid_small(N, K, 7 * N + K)
    yobs = np.random.default_rng(N).standard_normal(N).astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    td, Ad, wd, pd, yd = d(t), d(A), d(w), d(phi), d(yobs)
    nb = _capi.sinusoid_f32_residual_workspace_bytes(N)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    r = torch.empty_like(td)
    loss = torch.empty(1, device="cuda")
    _capi.sinusoid_f32_residual(td, yd, Ad, wd, pd, r, loss, ws, nb, N, K)
    torch.cuda.synchronize()
    y_or = oracle.sinusoid_forward(t, A, w, phi, threads=oracle.default_threads()) if K else \
        np.zeros(N, np.float32)
    r_or = (y_or - yobs).astype(np.float32)
    assert_bit_exact(r.cpu().numpy(), r_or, "residual N=%d K=%d" % (N, K))
    sq = r_or.astype(np.float64) ** 2
    exact = 0.5 * float(sq.sum())
    blocks = _capi.sinusoid_f32_residual_workspace_bytes(N) // 4
    depth = 8 + 8 + -(-blocks // 256) + 8 + 2
    assert abs(float(loss.cpu()[0]) - exact) <= depth * U * 0.5 * float(sq.sum()) * 1.001
    # in place: r over y_obs
    yd2 = d(yobs)
    _capi.sinusoid_f32_residual(td, yd2, Ad, wd, pd, yd2, loss, ws, nb, N, K)
    torch.cuda.synchronize()
    assert_bit_exact(yd2.cpu().numpy(), r_or, "residual in place N=%d" % N)
    # in place: r over t
    td2 = d(t)
    _capi.sinusoid_f32_residual(td2, yd, Ad, wd, pd, td2, loss, ws, nb, N, K)
    torch.cuda.synchronize()
    assert_bit_exact(td2.cpu().numpy(), r_or, "residual in place over t N=%d" % N)


@pytest.mark.parametrize("N,K", [(1, 1), (2047, 3), (2048, 64), (4099, 64), (300000, 64),
                                 (5000, 130), (3000, 0), (0, 5)])
def test_fit_step_matches_the_two_pass_path(torch_dev, N, K):
    """The one-pass fit step gives the same gradient bits as the forward
    kernel's residual followed by the adjoint kernel, and a loss within the
    rounding bound of its own fixed-order sums of the oracle's residual."""
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    t, A, w, phi = _sinusoid_small(N, K, 3 * N + K + 1)
    yobs = np.random.default_rng(N + 7).standard_normal(N).astype(np.float32)
    d = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda() if a.size else torch.empty(0, device="cuda")  # noqa: E731
    td, Ad, wd, pd, yd = d(t), d(A), d(w), d(phi), d(yobs)
    Kk = max(K, 1)
    g1 = [torch.full((Kk,), float("nan"), device="cuda") for _ in range(3)]
    loss1 = torch.full((1,), float("nan"), device="cuda")
    nb = _capi.sinusoid_f32_fit_step_workspace_bytes(N, K)
    ws = torch.empty(max(nb, 4), dtype=torch.uint8, device="cuda")
    _capi.sinusoid_f32_fit_step(td, yd, Ad, wd, pd, loss1, *g1, ws, nb, N=N, K=K)
    # the two-pass path
    r = torch.empty(max(N, 1), device="cuda")
    loss2 = torch.empty(1, device="cuda")
    g2 = [torch.full((Kk,), float("nan"), device="cuda") for _ in range(3)]
    nb_r = _capi.sinusoid_f32_residual_workspace_bytes(N)
    nb_b = _capi.sinusoid_f32_backward_workspace_bytes(N, K)
    ws2 = torch.empty(max(nb_r, nb_b, 4), dtype=torch.uint8, device="cuda")
    _capi.sinusoid_f32_residual(td, yd, Ad, wd, pd, r, loss2, ws2, nb_r, N, K)
    if K > 0:
        _capi.sinusoid_f32_backward(td, r, Ad, wd, pd, *g2, ws2, nb_b, N, K)
    torch.cuda.synchronize()
    for a, b, name in zip(g1, g2, ("gA", "gw", "gphi")):
        if K > 0:
            assert torch.equal(a[:K].view(torch.int32), b[:K].view(torch.int32)), (name, N, K)
    y_or = oracle.sinusoid_forward(t, A, w, phi, threads=oracle.default_threads()) if K and N else \
        np.zeros(N, np.float32)
    r_or = (y_or - yobs).astype(np.float32).astype(np.float64)
    sq = r_or ** 2
    exact = 0.5 * float(sq.sum())
    depth = 2 + 10 + -(-max(1, -(-N // 2048)) // 256) + 8 + 2
    assert abs(float(loss1.cpu()[0]) - exact) <= depth * U * 0.5 * float(sq.sum()) * 1.001 + 0.0, (N, K)
    if N == 0:
        assert float(loss1.cpu()[0]) == 0.0


def test_fit_step_deterministic(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    t, A, w, phi = _sinusoid_small(100000, 64, 19)
    yobs = np.random.default_rng(5).standard_normal(t.size).astype(np.float32)
    d = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    args = [d(t), d(yobs), d(A), d(w), d(phi)]
    nb = _capi.sinusoid_f32_fit_step_workspace_bytes(t.size, A.size)
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    outs = []
    for _ in range(3):
        o = [torch.empty(1, device="cuda")] + [torch.empty(64, device="cuda") for _ in range(3)]
        _capi.sinusoid_f32_fit_step(*args, *o, ws, nb)
        torch.cuda.synchronize()
        outs.append([v.cpu() for v in o])
    for o in outs[1:]:
        for a, b in zip(outs[0], o):
            assert torch.equal(a.view(torch.int32), b.view(torch.int32))


def test_sinusoid_residual_empty(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi
    A = torch.ones(3, device="cuda")
    loss = torch.full((1,), 7.0, device="cuda")
    ws = torch.empty(4, dtype=torch.uint8, device="cuda")
    _capi.sinusoid_f32_residual(0, 0, A, A, A, 0, loss, ws, 4, N=0, K=3)
    torch.cuda.synchronize()
    assert float(loss.cpu()[0]) == 0.0


def test_sinusoid_deterministic(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd.autograd import sinusoid_loss_and_grads
    t, A, w, phi = _sinusoid_small(100000, 64, 9)
    d = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    yobs = d(np.random.default_rng(2).standard_normal(t.size).astype(np.float32))
    first = [v.cpu() for v in sinusoid_loss_and_grads(d(t), yobs, d(A), d(w), d(phi))]
    for _ in range(3):
        again = [v.cpu() for v in sinusoid_loss_and_grads(d(t), yobs, d(A), d(w), d(phi))]
        for a, b in zip(first, again):
            assert torch.equal(a, b)


def test_sinusoid_autograd_matches_kernels(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd.autograd import sinusoid, sinusoid_loss_and_grads
    t, A, w, phi = _sinusoid_small(50000, 64, 12)
    d = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    yobs = d(np.random.default_rng(3).standard_normal(t.size).astype(np.float32))
    Ap, wp, pp = (d(a).requires_grad_(True) for a in (A, w, phi))
    y = sinusoid(d(t), Ap, wp, pp)
    loss = 0.5 * ((y - yobs) ** 2).sum()
    loss.backward()
    L, gA, gw, gp = sinusoid_loss_and_grads(d(t), yobs, d(A), d(w), d(phi))
    # same kernels, same residual: identical gradients
    assert torch.equal(Ap.grad, gA) and torch.equal(wp.grad, gw) and torch.equal(pp.grad, gp)
    with pytest.raises(NotImplementedError):
        sinusoid(d(t).requires_grad_(True), d(A), d(w), d(phi)).sum().backward()


@pytest.mark.slow
def test_sinusoid_fitting_workload_sampled(torch_dev):
    """N = 4,194,304 samples, K = 64, the fitting problem's data: forward
    bit-exact on a sample of samples; adjoint within the rounding bound for a
    sample of frequencies (the oracle evaluates each one exactly), and within
    the error-model bound of the exact-angle double-precision gradient."""
    torch = torch_dev
    from paper_cs_0406049_amd import workloads
    from paper_cs_0406049_amd.autograd import sinusoid_loss_and_grads
    from paper_cs_0406049_amd import _capi
    p = workloads.sinusoid_problem()
    d = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    td, Ad, wd, pd, yd = d(p.t), d(p.A), d(p.w), d(p.phi), d(p.y_obs)
    y = torch.empty_like(td)
    _capi.sinusoid_f32_forward(td, Ad, wd, pd, y)
    L, gA, gw, gp = sinusoid_loss_and_grads(td, yd, Ad, wd, pd)
    torch.cuda.synchronize()
    yh = y.cpu().numpy()
    idx = np.random.default_rng(0).choice(p.t.size, 20000, replace=False)
    yo = oracle.sinusoid_forward(p.t[idx], p.A, p.w, p.phi)
    assert_bit_exact(yh[idx], yo, "fitting forward (sample)")
    r = (yh - p.y_obs).astype(np.float32)
    ks = [0, 17, 40, 63]
    ref = oracle.sinusoid_adjoint(p.t, r, p.A[ks], p.w[ks], p.phi[ks])
    got = {"gA": gA.cpu().numpy()[ks], "gw": gw.cpu().numpy()[ks], "gphi": gp.cpu().numpy()[ks]}
    for key, absk in (("gA", "abs_A"), ("gw", "abs_w"), ("gphi", "abs_phi")):
        err = np.abs(got[key].astype(np.float64) - ref[key])
        assert np.all(err <= _adjoint_bound(p.t.size, ref[absk]) + np.abs(ref[key]) * U), key
        log("fitting %s: max err / |term| sum = %.3g" % (key, (err / ref[absk]).max()))
    # exact angles in double precision with the system sine: the difference is
    # bounded by sum_i |r_i| (E_pair(theta32) + |theta32 - theta64|) (times
    # |A_k|, and t_i for w) plus the rounding bound above
    t64, r64 = p.t.astype(np.float64), r.astype(np.float64)
    kinv = 1.0 / (2 * math.pi)
    for j, k in enumerate(ks):
        th64 = float(p.w[k]) * t64 + float(p.phi[k])
        th32 = th64.astype(np.float32)
        ulp_th = (np.nextafter(np.abs(th32), np.float32(np.inf)) - np.abs(th32)).astype(np.float64)
        x1 = np.abs((th32 * np.float32(kinv)).astype(np.float32))
        ulp_x1 = (np.nextafter(x1, np.float32(np.inf)) - x1).astype(np.float64)
        e = 4.95e-7 + np.abs(th64) * 4.1e-8 + math.pi * ulp_x1 + ulp_th
        a = abs(float(p.A[k]))
        for key, exact, wgt in (("gA", np.dot(r64, np.sin(th64)), np.abs(r64)),
                                ("gphi", float(p.A[k]) * np.dot(r64, np.cos(th64)), a * np.abs(r64)),
                                ("gw", float(p.A[k]) * np.dot(r64 * t64, np.cos(th64)),
                                 a * np.abs(r64) * t64)):
            bound = float(np.dot(wgt, e)) + _adjoint_bound(p.t.size, ref["abs_" + key[1:]][j]) \
                + abs(exact) * U
            assert abs(float(got[key][j]) - exact) <= bound, (key, k)
