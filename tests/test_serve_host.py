"""The request server's scheduling on the host, with the simulated executor
(no device work): admission by budget, arrival order, continuous batching
and overlap, latency accounting, failure and shutdown paths."""
import ctypes
import time

import numpy as np
import pytest

from paper_cs_0406049_amd import _capi, serve
from paper_cs_0406049_amd import build as hipbuild

FAKE = 1 << 33  # input addresses are never dereferenced by the simulated executor


@pytest.fixture(scope="module", autouse=True)
def _lib():
    if not hipbuild.is_built():
        hipbuild.build()
    _capi.lib()


def sim(**kw):
    kw.setdefault("executor", serve.EXEC_SIM)
    return serve.Server(**kw)


def drain(srv, count, timeout=10.0):
    out = []
    t_end = time.time() + timeout
    while len(out) < count and time.time() < t_end:
        out += srv.poll(256, 0.05)
    return out


def test_config_validation():
    for bad in (dict(budget_bytes=-1), dict(max_inflight=17), dict(mode=2), dict(executor=5),
                dict(arith=3), dict(max_batch_requests=-2)):
        with pytest.raises(_capi.SincosError) as e:
            sim(**bad)
        assert e.value.status == _capi.EINVAL
    # stream_per_slot takes 0 or 1 only (the binding passes a bool)
    cfg = _capi.ServerConfig(executor=serve.EXEC_SIM, stream_per_slot=2)
    h = ctypes.c_void_p()
    assert _capi.lib().sincos_server_create(ctypes.byref(cfg), ctypes.byref(h)) == _capi.EINVAL
    assert not h.value


def test_submit_validation_and_budget_reject():
    with sim(budget_bytes=12_000) as s:
        with pytest.raises(_capi.SincosError) as e:
            s.submit(FAKE, 1001)
        assert e.value.status == _capi.EBUDGET
        for bad in ((FAKE, 0), (FAKE, -5), (0, 10), (FAKE + 2, 10)):
            with pytest.raises(_capi.SincosError):
                s.submit(*bad)
        rid = s.submit(FAKE, 1000)
        got = drain(s, 1)
        assert len(got) == 1 and got[0].id == rid and got[0].status == _capi.OK
        assert got[0].s and got[0].c and got[0].c - got[0].s >= 4000
        s.release(rid)
        with pytest.raises(_capi.SincosError):
            s.release(rid)


def test_budget_bounds_admission_and_release_frees_it():
    """Budget for 3 requests: the 4th waits until one is released."""
    n = 1000
    with sim(budget_bytes=3 * 12 * n, sim_batch_ns=1000) as s:
        ids = [s.submit(FAKE + 4096 * j, n, tag=j) for j in range(4)]
        first = drain(s, 3, timeout=2.0)
        assert sorted(c.tag for c in first) == [0, 1, 2]
        assert not s.poll(16, 0.2)           # 4th still blocked on the budget
        st = s.stats()
        assert st["budget_in_use"] == 3 * 12 * n and st["admitted"] == 3
        s.release(first[0].id)
        last = drain(s, 1, timeout=2.0)
        assert [c.tag for c in last] == [3]
        assert s.stats()["budget_peak"] == 3 * 12 * n
        for c in first[1:] + last:
            s.release(c.id)
        assert s.stats()["budget_in_use"] == 0
        assert ids[3] == last[0].id


def test_arrival_order_no_overtaking():
    """A large head request blocked on the budget is not overtaken."""
    with sim(budget_bytes=12 * 10_000, sim_batch_ns=2000, auto_release=True) as s:
        s.submit(FAKE, 9000, tag=0)
        s.submit(FAKE, 9000, tag=1)          # must wait for tag 0
        s.submit(FAKE, 100, tag=2)           # fits now, but arrives after tag 1
        got = drain(s, 3)
        admit = {c.tag: c.t_admit_ns for c in got}
        assert admit[0] < admit[1] <= admit[2]


def test_continuous_batching():
    """Requests arriving while batches run join later batches."""
    # 300 arrivals 100 us apart (a 30 ms stream), 2 ms batches, 3 in flight:
    # about one launch per 0.7 ms with ~7 requests each.  The bounds hold even
    # when the host delays the scheduler thread by milliseconds (a busy machine
    # gives fewer, larger batches, not fewer than a handful).
    count = 300
    arr = np.arange(count, dtype=np.int64) * 100_000
    ns = np.full(count, 5000, np.int64)
    with sim(max_inflight=3, sim_batch_ns=2_000_000, auto_release=True) as s:
        out = s.replay([FAKE] * count, ns, arr)
        st = s.stats()
    lat = out["t_complete_ns"] - out["t_submit_ns"]
    info = (st, int(out["batch_requests"].max()), float(np.percentile(lat, 99)))
    assert np.all(out["status"] == 0)
    assert 3 < st["batches"] < count / 2, info             # batched, and continuously
    assert out["batch_requests"].max() > 1, info
    assert np.all(lat > 0)
    assert np.all(out["t_submit_ns"] <= out["t_admit_ns"])
    assert np.all(out["t_admit_ns"] <= out["t_launch_ns"])
    assert np.all(out["t_launch_ns"] < out["t_complete_ns"])
    # latency is bounded by batch times, not by the whole 30 ms stream
    assert np.percentile(lat, 99) < 24_000_000, info


def test_batches_overlap_up_to_max_inflight():
    """With work for several batches waiting, one scheduler trip fills every
    free slot: max_inflight batches run at once."""
    count = 60
    with sim(max_inflight=3, max_batch_requests=5, sim_batch_ns=5_000_000,
             auto_release=True) as s:
        out = s.replay([FAKE] * count, np.full(count, 5000, np.int64),
                       np.zeros(count, np.int64))
        st = s.stats()
    assert np.all(out["status"] == 0)
    assert st["inflight_peak"] == 3, st
    assert out["batch_requests"].max() <= 5


def test_batch_caps():
    with sim(max_batch_requests=7, max_inflight=1, sim_batch_ns=50_000, auto_release=True) as s:
        out = s.replay([FAKE] * 100, np.full(100, 10, np.int64), np.zeros(100, np.int64))
        assert out["batch_requests"].max() <= 7
    with sim(max_batch_elems=2500, max_inflight=1, sim_batch_ns=50_000, auto_release=True) as s:
        out = s.replay([FAKE] * 60, np.full(60, 1000, np.int64), np.zeros(60, np.int64))
        assert out["batch_requests"].max() <= 2


def test_size_split_never_mixes_classes_in_a_batch():
    """With a size split, a batch holds only requests above the split or
    only requests at or below it; the oldest waiting request picks the class
    and each class keeps its arrival order.  split_elems -1 mixes them."""
    sizes = np.array([5000, 10, 20, 6000, 30, 7000, 40, 50, 8000, 60] * 6, np.int64)
    for split, mixed_ok in ((1000, False), (-1, True)):
        with sim(max_inflight=1, sim_batch_ns=200_000, auto_release=True,
                 split_elems=split) as s:
            # the first request occupies the one slot while the rest queue up
            out = s.replay([FAKE] * sizes.size, sizes, np.zeros(sizes.size, np.int64))
        assert np.all(out["status"] == 0)
        mixed = False
        for t in np.unique(out["t_launch_ns"]):
            members = np.flatnonzero(out["t_launch_ns"] == t)
            big = sizes[members] > 1000
            mixed |= bool(big.any() and not big.all())
            # within a batch, requests keep their arrival order
            assert np.all(np.diff(out["t_submit_ns"][members]) >= 0)
        assert mixed == mixed_ok, (split, mixed)
        if not mixed_ok:
            # each class is launched in arrival order
            for cls in (sizes > 1000, sizes <= 1000):
                assert np.all(np.diff(out["t_launch_ns"][cls]) >= 0)
    with pytest.raises(_capi.SincosError):
        sim(split_elems=-2)


def test_per_request_mode_one_launch_each():
    with sim(mode=serve.MODE_PER_REQUEST, sim_batch_ns=5000, auto_release=True) as s:
        out = s.replay([FAKE] * 50, np.full(50, 100, np.int64), np.zeros(50, np.int64))
        assert np.all(out["batch_requests"] == 1)
        assert s.stats()["batches"] == 50


def test_failed_batches_error_only_their_requests():
    with sim(sim_fail_every=3, max_inflight=1, max_batch_requests=1, sim_batch_ns=1000,
             auto_release=True) as s:
        with pytest.raises(_capi.SincosError):
            s.replay([FAKE] * 30, np.full(30, 10, np.int64), np.zeros(30, np.int64))
        st = s.stats()
        assert st["failed"] == 10 and st["completed"] == 20
        assert st["budget_in_use"] == 0


def test_failed_request_memory_is_returned_without_release():
    with sim(sim_fail_every=1, sim_batch_ns=1000) as s:
        rid = s.submit(FAKE, 1000)
        c = drain(s, 1)[0]
        assert c.id == rid and c.status == _capi.EHIP and not c.s
        assert s.stats()["budget_in_use"] == 0


def test_shutdown_cancels_pending_and_drains():
    s = sim(budget_bytes=12 * 1000, sim_batch_ns=200_000)
    for j in range(5):
        s.submit(FAKE, 1000, tag=j)       # only one fits at a time
    time.sleep(0.02)
    lib = _capi.lib()
    h = s._h
    assert lib.sincos_server_destroy(h) == _capi.OK
    s._h = None


def test_output_placement_keeps_the_input_phase():
    """Outputs start at the input's offset modulo 16 bytes (float4 path)."""
    with sim() as s:
        for ph in (0, 4, 8, 12):
            rid = s.submit(FAKE + ph, 1000 + ph)
            c = drain(s, 1)[0]
            assert c.s % 16 == ph and c.c % 16 == ph and c.c >= c.s + 4 * c.n
            s.release(rid)


def test_latency_summary():
    comp = np.zeros(4, serve.COMPLETION_DTYPE)
    comp["t_submit_ns"] = [0, 10, 20, 30]
    comp["t_complete_ns"] = [1000, 2010, 3020, 4030]
    comp["n"] = 10
    comp["batch_requests"] = 2
    s = serve.latency_summary(comp)
    assert s["p50_us"] == pytest.approx(2.5) and s["max_us"] == pytest.approx(4.0)
    assert s["elements"] == 40 and s["span_s"] == pytest.approx(4.03e-6)


def test_autotune_cache_keys_and_candidates(tmp_path):
    from paper_cs_0406049_amd import autotune
    k1 = autotune.cache_key("gfx950", 256, 4096, 453_000_000, 0, 0)
    k2 = autotune.cache_key("gfx950", 256, 4000, 300_000_000, 0, 0)
    k3 = autotune.cache_key("gfx950", 256, 4096, 453_000_000, 1, 0)
    assert k1 == k2 and k1 != k3
    cands = list(autotune.candidates(256))
    persistent = [w for w in autotune.WAVES_PER_CU if w]
    capped = [(b, cap) for b in autotune.BLOCKS for cap in autotune.WAVE_CAPS
              if autotune.lds_for_cap(b, cap) is not None]
    assert len(cands) == len(autotune.UNROLLS) * (len(autotune.BLOCKS) * len(persistent) +
                                                 len(capped))
    assert len(set(cands)) == len(cands)
    assert all(b % 64 == 0 and u in (1, 2, 4, 8) and g >= 1 and (l == -1 or 0 < l <= 65536)
               for b, u, g, l in cands)
    # an LDS reservation holds a CU to at least the capped number of waves
    for b, u, g, l in cands:
        if l > 0:
            assert g == autotune.COVER
            waves = (autotune.LDS_PER_CU // l) * (b // 64)
            assert min(autotune.WAVE_CAPS[1:]) <= waves <= 2 * max(autotune.WAVE_CAPS), (b, l)
    p = str(tmp_path / "t.json")
    autotune.save_cache({k1: {"shape": [256, 4, 2048]}}, p)
    assert autotune.load_cache(p)[k1]["shape"] == [256, 4, 2048]
    assert autotune.load_cache(str(tmp_path / "missing.json")) == {}


def test_replay_rejects_mismatched_tables():
    with sim(auto_release=True) as s:
        with pytest.raises(ValueError):
            s.replay([FAKE] * 3, np.full(4, 100, np.int64), np.zeros(4, np.int64))


def test_submit_on_with_the_simulated_executor():
    """submit_on takes the same arguments as submit plus a stream; a simulated
    server has no device work to wait for and ignores the stream."""
    import ctypes
    with sim(budget_bytes=1 << 20) as s:
        rid = ctypes.c_int64()
        assert _capi.lib().sincos_server_submit_on(s._h, FAKE, 1000, 7, None,
                                                   ctypes.byref(rid)) == _capi.OK
        for bad_x, bad_n in ((0, 10), (FAKE + 2, 10), (FAKE, 0)):
            assert _capi.lib().sincos_server_submit_on(s._h, bad_x, bad_n, 0, None,
                                                       ctypes.byref(rid)) == _capi.EINVAL
        assert _capi.lib().sincos_server_submit_on(s._h, FAKE, 1 << 20, 0, None,
                                                   ctypes.byref(rid)) == _capi.EBUDGET
        got = drain(s, 1)
        assert len(got) == 1 and got[0].tag == 7 and got[0].status == _capi.OK
