"""The ragged form's autotuner and its pre-marshalled one-shot path on the GPU.

The autotuner times every candidate launch shape (block, unroll, grid, LDS
reservation) on the 4096-array workload, then the fastest few again in
interleaved rounds; its choice must come from the candidate set, and the plan built with that choice, launched through its
HIP graph, must be bit-exact against the oracle on every element.  A
one-shot call with a SegTable (tables marshalled once) must give the same
bits as the call with the tensor list."""
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


def test_autotuned_plan_on_the_full_workload_is_bit_exact(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, autotune, workloads
    lens, xs_h = workloads.ragged_batch()
    segs = []
    for xh in xs_h:
        x = torch.from_numpy(xh).cuda()
        segs.append((x, torch.empty_like(x), torch.empty_like(x)))
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    best, table = autotune.tune_ragged_table(segs, lens, reps=2)
    cands = list(autotune.candidates(cus))
    log("autotune: %d candidates timed, best %s at %.4f ms; slowest %.4f ms"
        % (len(table), best, table[0][0], table[-1][0]))
    assert tuple(best) in set(cands)
    assert len(table) == len(cands) and table[0][1] == best
    assert {sh for _, sh in table} == set(cands)
    fin, rest = table[:autotune.FINALISTS], table[autotune.FINALISTS:]
    assert fin == sorted(fin) and rest == sorted(rest)      # finalists by median, then the rest
    plan = _capi.RaggedPlan(segs, lens, launch=best)
    for _, s, c in segs:
        s.fill_(float("nan"))
        c.fill_(float("nan"))
    plan.graph_launch()
    torch.cuda.synchronize()
    flat_x = np.concatenate(xs_h)
    so, co = oracle.sincos(flat_x, 0, 0, threads=oracle.default_threads())
    sg = torch.cat([s for _, s, _ in segs]).cpu().numpy()
    assert_bit_exact(sg, so, "autotuned ragged sin", flat_x)
    del sg
    cg = torch.cat([c for _, _, c in segs]).cpu().numpy()
    assert_bit_exact(cg, co, "autotuned ragged cos", flat_x)
    log("autotuned plan %s: %d segments, %d elements bit-exact" % (best, len(lens), flat_x.size))
    plan.destroy()


def test_segtable_one_shot_matches_the_tensor_list(torch_dev):
    torch = torch_dev
    from paper_cs_0406049_amd import _capi, workloads
    lens = workloads.ragged_lengths(700, lo=1, hi=3e4, seed=11)
    lens[::97] = 0                                         # some empty segments
    rng = np.random.default_rng(12)
    segs = []
    for n in lens:
        x = torch.from_numpy(rng.uniform(-1e3, 1e3, int(n)).astype(np.float32)).cuda()
        segs.append((x, torch.full_like(x, float("nan")), torch.full_like(x, float("nan"))))
    _capi.sincos_f32_ragged(segs, lens)
    torch.cuda.synchronize()
    want = [(s.clone(), c.clone()) for _, s, c in segs]
    for make in (lambda: _capi.SegTable(segs, lens),
                 lambda: _capi.SegTable.from_pointers(
                     np.array([[x.data_ptr(), s.data_ptr(), c.data_ptr()] for x, s, c in segs],
                              np.uint64), lens)):
        table = make()
        for _, s, c in segs:
            s.fill_(float("nan"))
            c.fill_(float("nan"))
        _capi.sincos_f32_ragged(table)
        _capi.sincos_f32_ragged(table)                     # reusable
        torch.cuda.synchronize()
        for (s0, c0), (_, s, c) in zip(want, segs):
            assert torch.equal(s.view(torch.int32), s0.view(torch.int32))
            assert torch.equal(c.view(torch.int32), c0.view(torch.int32))
    with pytest.raises(ValueError):
        _capi.sincos_f32_ragged(_capi.SegTable(segs, lens), lens)
