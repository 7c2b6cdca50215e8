"""The C-ABI library on a machine with or without a GPU: it loads, exports
every symbol include/sincos.h declares, and rejects bad arguments on the host
before any HIP call.  Pointers here are fake addresses that are never
dereferenced: every case fails validation first (or is a no-op)."""
import ctypes
import os
import re

import pytest

from paper_cs_0406049_amd import _capi, build as hipbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sincos.h")


@pytest.fixture(scope="module")
def L():
    if not hipbuild.is_built():
        hipbuild.build()
    return _capi.lib()


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"SINCOS_API\s+[\w\s\*]+?\b(\w+)\s*\(", text)))


def test_every_declared_symbol_is_exported(L):
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_capi._SIGNATURES), "binding and header disagree"


@pytest.mark.parametrize("lib_name,name", [("sqrt_rn_check", "sqrt_rn_check"),
                                           ("sqrt_rn_check", "sqrt_rn_finite_check"),
                                           ("rcp_rn_check", "rcp_rn_check"),
                                           ("lockstep_check", "lockstep_check")])
def test_check_helpers_are_built_and_export_their_entries(L, lib_name, name):
    """The GPU tests' square-root, reciprocal and lockstep check libraries (built beside
    the tests by __graft_entry__.build()) export their entry points."""
    import subprocess
    lib = os.path.join(ROOT, "tests", "native", "lib%s.so" % lib_name)
    if not os.path.exists(lib):
        hipbuild.build_test_helpers()
    out = subprocess.run(["nm", "-D", "--defined-only", lib], capture_output=True,
                         text=True).stdout
    assert re.search(r"\bT %s$" % name, out, re.M), out


def test_only_declared_symbols_are_exported(L):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", _capi.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    assert exported == set(declared_functions()), exported ^ set(declared_functions())


def test_version(L):
    assert "gfx950" in _capi.version()


BASE = 1 << 32  # fake, 256-byte aligned addresses


def st(rc):
    return rc, _capi.last_error()


def test_plain_validation(L):
    f = L.sincos_f32
    assert f(None, None, None, 0, None) == _capi.OK
    assert st(f(None, None, None, -1, None))[0] == _capi.EINVAL
    assert st(f(None, BASE, BASE + 4096, 4, None))[0] == _capi.EINVAL
    assert st(f(BASE + 1, BASE + 4096, BASE + 8192, 4, None))[0] == _capi.EINVAL  # misaligned
    assert st(f(BASE, BASE + 4096, BASE + 4096, 4, None))[0] == _capi.EOVERLAP    # s == c
    assert st(f(BASE, BASE + 4096, BASE + 4096 + 8, 4, None))[0] == _capi.EOVERLAP  # s, c overlap
    assert st(f(BASE, BASE + 8, BASE + 8192, 4, None))[0] == _capi.EOVERLAP       # x partly s
    assert st(f(BASE + 8, BASE, BASE + 8192, 4, None))[0] == _capi.EOVERLAP
    assert st(f(BASE, BASE + 8192, BASE + 4, 4, None))[0] == _capi.EOVERLAP       # x partly c
    ex = L.sincos_f32_ex
    assert ex(BASE, BASE + 4096, BASE + 8192, 4, 3, 0, None, None) == _capi.EINVAL
    assert ex(BASE, BASE + 4096, BASE + 8192, 4, 0, 2, None, None) == _capi.EINVAL
    for bad in ((96, 4, 0), (2048, 4, 0), (256, 3, 0), (256, 4, -1)):
        rc = ex(BASE, BASE + 4096, BASE + 8192, 4, 0, 0, ctypes.byref(_capi.Launch(*bad, 0)), None)
        assert rc == _capi.EINVAL, bad
    assert "launch" in _capi.last_error()


def test_in_place_is_accepted_by_validation(L):
    """x == s (or x == c) passes the argument checks: the call then either
    runs (GPU present) or reports the missing device, never EOVERLAP."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("covered by the GPU tests")
    for args in ((BASE, BASE, BASE + 4096), (BASE, BASE + 4096, BASE)):
        assert L.sincos_f32(*args, 4, None) == _capi.ENODEV
    assert "device" in _capi.last_error()


def seg_tables(segs, lens):
    S = (_capi.Seg * len(segs))(*[_capi.Seg(*t) for t in segs])
    N = (ctypes.c_int64 * len(lens))(*lens)
    return S, N


def test_ragged_validation(L):
    f = L.sincos_f32_ragged
    S, N = seg_tables([(BASE, BASE + 4096, BASE + 8192)], [4])
    assert f(S, N, 0, None) == _capi.OK
    assert f(S, N, -1, None) == _capi.EINVAL
    assert f(None, N, 1, None) == _capi.EINVAL
    S, N = seg_tables([(BASE, BASE + 4096, BASE + 8192)], [-3])
    assert f(S, N, 1, None) == _capi.EINVAL
    assert "segment 0" in _capi.last_error()
    # outputs of two segments overlap
    S, N = seg_tables([(BASE, BASE + 4096, BASE + 8192), (BASE + 100000, BASE + 8192 + 8, BASE + 200000)],
                      [4, 4])
    assert f(S, N, 2, None) == _capi.EOVERLAP
    # input of one segment overlaps an output of another
    S, N = seg_tables([(BASE, BASE + 4096, BASE + 8192), (BASE + 4096, BASE + 20000, BASE + 30000)],
                      [4, 4])
    assert f(S, N, 2, None) == _capi.EOVERLAP
    # shared inputs, disjoint outputs, and in-place segments pass validation
    import torch
    if not torch.cuda.is_available():
        S, N = seg_tables([(BASE, BASE + 4096, BASE + 8192), (BASE, BASE + 12288, BASE + 16384),
                           (BASE + 20480, BASE + 20480, BASE + 24576)], [4, 4, 4])
        assert f(S, N, 3, None) == _capi.ENODEV
        # zero-length segments are ignored, whatever their pointers
        S, N = seg_tables([(0, 0, 0), (BASE, BASE + 4096, BASE + 8192)], [0, 4])
        assert f(S, N, 2, None) == _capi.ENODEV


def test_plan_validation(L):
    h = ctypes.c_void_p()
    S, N = seg_tables([(BASE, BASE + 4096, BASE + 4096)], [4])
    assert L.sincos_ragged_plan_create(S, N, 1, 0, 0, None, ctypes.byref(h)) == _capi.EOVERLAP
    assert not h.value
    assert L.sincos_ragged_plan_create(S, N, 1, 0, 0, None, None) == _capi.EINVAL
    assert L.sincos_ragged_plan_launch(None, None) == _capi.EINVAL
    assert L.sincos_ragged_plan_graph_launch(None, None) == _capi.EINVAL
    assert L.sincos_ragged_plan_destroy(None) == _capi.OK


def test_backward_validation(L):
    f = L.sincos_f32_backward
    assert f(None, None, None, None, None, 0, None) == _capi.OK
    assert f(BASE, BASE + 4096, None, None, BASE + 8192, -1, None) == _capi.EINVAL
    assert f(BASE, None, None, None, BASE + 8192, 4, None) == _capi.EINVAL
    assert f(BASE, BASE + 4096, None, None, BASE + 4, 4, None) == _capi.EOVERLAP
    assert f(BASE, BASE + 4096, BASE + 8192 + 4, None, BASE + 8192, 4, None) == _capi.EOVERLAP


def test_sinusoid_validation_and_workspace(L):
    assert L.sinusoid_f32_forward(None, -1, None, None, None, 0, None, None) == _capi.EINVAL
    assert L.sinusoid_f32_forward(BASE, 4, None, None, None, 3, BASE + 4096, None) == _capi.EINVAL
    assert L.sinusoid_f32_forward(None, 0, BASE, BASE, BASE, 3, None, None) == _capi.OK
    wb = L.sinusoid_f32_backward_workspace_bytes
    assert wb(-1, 4) == -1
    assert wb(4_194_304, 64) == 2048 * 3 * 64 * 4      # one partial per 2048 samples and lane
    assert wb(1025, 65) == 1 * 3 * 128 * 4
    assert wb(8193, 1) == 5 * 3 * 64 * 4
    rc = L.sinusoid_f32_backward(BASE, BASE, (1 << 31) * 2048 + 1, BASE, BASE, BASE, 4, BASE, BASE,
                                 BASE, BASE, 1 << 40, None)
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()
    rc = L.sinusoid_f32_backward(BASE, BASE + 4096, 4096, BASE + 8192, BASE + 8192, BASE + 8192, 64,
                                 BASE + 9000, BASE + 10000, BASE + 11000, BASE + 20000, 16, None)
    assert rc == _capi.EINVAL and "workspace" in _capi.last_error()


def test_sinusoid_aliasing_and_alignment(L):
    """The sinusoid calls reject outputs that overlap their inputs, the
    parameters or each other, and misaligned arrays, before any HIP call."""
    t, y, A, w, p = BASE, BASE + 65536, BASE + 2 * 65536, BASE + 3 * 65536, BASE + 4 * 65536
    fwd = L.sinusoid_f32_forward
    assert fwd(t, 16, A, w, p, 8, A + 4, None) == _capi.EOVERLAP           # y over A
    assert "A" in _capi.last_error()
    assert fwd(t, 16, A, w, p, 8, p - 8, None) == _capi.EOVERLAP           # y over phi
    assert fwd(t, 16, A, w, p, 8, t + 4, None) == _capi.EOVERLAP           # y partly t
    assert fwd(t + 2, 16, A, w, p, 8, y, None) == _capi.EINVAL             # misaligned t
    assert fwd(t, 16, A, w + 1, p, 8, y, None) == _capi.EINVAL             # misaligned w
    res = L.sinusoid_f32_residual
    yo, r, loss, ws = BASE + 5 * 65536, BASE + 6 * 65536, BASE + 7 * 65536, BASE + 8 * 65536
    assert res(t, yo, 16, A, w, p, 8, r, loss, A, 64, None) == _capi.EOVERLAP   # ws over A
    assert res(t, yo, 16, A, w, p, 8, r, loss, r + 16, 64, None) == _capi.EOVERLAP  # ws over r
    assert res(t, yo, 16, A, w, p, 8, r, w + 4, ws, 64, None) == _capi.EOVERLAP  # loss in w
    assert res(t, yo, 16, A, w, p, 8, r, loss, ws + 2, 64, None) == _capi.EINVAL
    bwd = L.sinusoid_f32_backward
    gA, gw, gp = BASE + 9 * 65536, BASE + 10 * 65536, BASE + 11 * 65536
    need = L.sinusoid_f32_backward_workspace_bytes(16, 8)
    ok = (t, y, 16, A, w, p, 8, gA, gw, gp, ws, need, None)

    def bad(**kw):
        names = ("t", "g", "N", "A", "w", "phi", "K", "gA", "gw", "gphi", "ws", "wsb", "st")
        args = dict(zip(names, ok))
        args.update(kw)
        return bwd(*[args[n] for n in names])
    assert bad(gA=A) == _capi.EOVERLAP                 # in-place gradient into A
    assert bad(gw=gA + 4) == _capi.EOVERLAP            # gw overlaps gA
    assert bad(gphi=t + 8) == _capi.EOVERLAP           # gphi inside t
    assert bad(ws=gp) == _capi.EOVERLAP                # workspace over gphi
    assert bad(ws=y) == _capi.EOVERLAP                 # workspace over g
    assert bad(gA=gA + 2) == _capi.EINVAL              # misaligned
    assert bad(g=y + 1) == _capi.EINVAL


def test_sinusoid_residual_validation(L):
    f = L.sinusoid_f32_residual
    wb = L.sinusoid_f32_residual_workspace_bytes
    assert wb(-1) == -1
    assert wb(4_194_304) == 2048 * 4               # one float per 2048-sample workgroup
    assert wb(1) == 4 and wb(0) == 4
    assert wb(1 << 40) == (1 << 20) * 4            # the grid is capped; the kernel strides
    t, yo, r, loss, ws = BASE, BASE + 65536, BASE + 2 * 65536, BASE + 3 * 65536, BASE + 4 * 65536
    prm = (BASE + 5 * 65536,) * 3
    assert f(t, yo, -1, *prm, 4, r, loss, ws, 64, None) == _capi.EINVAL
    assert f(t, yo, 16, *prm, 4, r, None, ws, 64, None) == _capi.EINVAL          # null loss
    assert f(t, None, 16, *prm, 4, r, loss, ws, 64, None) == _capi.EINVAL        # null y_obs
    assert f(t, yo, 16, *prm, 4, t + 4, loss, ws, 64, None) == _capi.EOVERLAP    # r partly t
    assert f(t, yo, 16, *prm, 4, r, r + 8, ws, 64, None) == _capi.EOVERLAP       # loss inside r
    rc = f(t, yo, 16, *prm, 4, r, loss, ws, 0, None)
    assert rc == _capi.EINVAL and "workspace" in _capi.last_error()
    assert f(t, yo, 16, None, None, None, 4, r, loss, ws, 64, None) == _capi.EINVAL


def test_copy_ceiling_validation(L):
    f = L.sincos_copy_ceiling_f32
    assert f(BASE, BASE + 4096, BASE + 8192, 6, None, None) == _capi.EINVAL
    assert f(BASE + 4, BASE + 4096, BASE + 8192, 4, None, None) == _capi.EINVAL
    assert f(BASE, BASE, BASE + 8192, 4, None, None) == _capi.EOVERLAP


def test_pair_ceiling_validation(L):
    f = L.sincos_pair_ceiling_f32
    assert f(None, None, 0, 4, None) == _capi.OK
    assert f(BASE, BASE + 4096, -1, 4, None) == _capi.EINVAL
    assert f(BASE, BASE + 4096, 4, -1, None) == _capi.EINVAL
    assert f(None, BASE + 4096, 4, 1, None) == _capi.EINVAL
    assert f(BASE + 2, BASE + 4096, 4, 1, None) == _capi.EINVAL
    assert f(BASE, BASE + 8, 4, 1, None) == _capi.EOVERLAP
    rc = f(BASE, BASE + 4096, (1 << 31) * 256, 1, None)
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """No silent fallback: without the built library the binding raises."""
    monkeypatch.setattr(_capi, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_capi, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        _capi.lib()


def test_tuning_round_trip_and_rejection(L):
    from paper_cs_0406049_amd import autotune
    builtin = {"plain": {"block": 64, "unroll": 1, "grid": 0, "lds": 7168},
               "ragged": {"block": 256, "unroll": 1, "grid": 0, "lds": 0}}
    try:
        _capi.set_tuning(None)
        assert _capi.get_tuning() == builtin
        autotune.install("ragged", (512, 2, 4096))
        want = {"plain": builtin["plain"],
                "ragged": {"block": 512, "unroll": 2, "grid": 4096, "lds": 0}}
        assert _capi.get_tuning() == want
        autotune.install("ragged", (64, 1, 1 << 30, 6656))
        assert _capi.get_tuning()["ragged"] == {"block": 64, "unroll": 1, "grid": 1 << 30,
                                                "lds": 6656}
        autotune.install("ragged", (64, 1, 1 << 30, -1))       # -1: no reservation
        assert _capi.get_tuning()["ragged"]["lds"] == 0
        # a form left out of the text gets the built-in shape back
        _capi.set_tuning({"plain": {"unroll": 4}})
        assert _capi.get_tuning() == {"plain": {"block": 64, "unroll": 4, "grid": 0, "lds": 7168},
                                      "ragged": builtin["ragged"]}
        _capi.set_tuning({"plain": (512, 2, 0, 0), "ragged": (1024, 8, 7, 65536)})
        kept = _capi.get_tuning()
        assert kept["ragged"]["lds"] == 65536 and kept["plain"]["lds"] == 0
        for bad in (b'{"plain": {"block": 100}}', b'{"plain": {"unroll": 3}}',
                    b'{"ragged": {"grid": -1}}', b'{"plan": {}}', b'{"plain": {"block": 1.5}}',
                    b'{"plain": {"block": 256', b'{} x', b'[]', b'{"plain": {"warps": 4}}',
                    b'{"plain": {"block": 99999999999}}', b'{"plain": {"grid": 2147483648}}',
                    b'{"plain": {"lds": -1}}', b'{"ragged": {"lds": 65537}}',
                    b'{"plain": {"lds": 1, "lds": 2}}', b''):
            assert L.sincos_set_tuning(bad) == _capi.EINVAL, bad
            assert "sincos_set_tuning" in _capi.last_error()
            assert _capi.get_tuning() == kept, bad
        # a short buffer is truncated with a terminator; the return is the full length
        n = L.sincos_get_tuning(None, 0)
        buf = ctypes.create_string_buffer(16)
        assert L.sincos_get_tuning(buf, 16) == n and len(buf.value) == 15
        assert L.sincos_set_tuning(b" { } ") == _capi.OK
        assert _capi.get_tuning() == builtin
    finally:
        _capi.set_tuning(None)


def test_huygens_validation(L):
    f = L.huygens_f32
    src = BASE + (1 << 20)          # 16-byte aligned source table
    args = lambda P, S, xo=BASE, yo=BASE + 65536, s=src, kk=1.0, LL=100.0, re=BASE + 2 * 65536, \
        im=BASE + 3 * 65536: (xo, yo, P, s, S, kk, LL, re, im, None)  # noqa: E731
    assert f(*args(0, 0)) == _capi.OK
    assert f(*args(-1, 4)) == _capi.EINVAL
    assert f(*args(4, -1)) == _capi.EINVAL
    assert f(*args(4, 4, xo=None)) == _capi.EINVAL
    assert f(*args(4, 4, s=None)) == _capi.EINVAL
    assert f(*args(4, 4, s=src + 4)) == _capi.EINVAL             # src not 16-byte aligned
    assert f(*args(4, 4, re=BASE + 2 * 65536 + 2)) == _capi.EINVAL
    for bad_L in (0.0, -1.0, float("inf"), float("nan")):
        assert f(*args(4, 4, LL=bad_L)) == _capi.EINVAL, bad_L
    assert f(*args(4, 4, im=BASE + 2 * 65536 + 8)) == _capi.EOVERLAP   # re and im overlap
    assert f(*args(4, 4, re=BASE + 8)) == _capi.EOVERLAP              # re overlaps xo
    assert f(*args(4, 4, im=src + 16)) == _capi.EOVERLAP              # im overlaps the sources
    rc = f(*args((1 << 31) * 256, 4))
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()


def test_interleaved_validation(L):
    f = L.sincos_f32_interleaved
    assert f(None, None, 0, 0, None) == _capi.OK
    assert f(BASE, BASE + 4096, -1, 0, None) == _capi.EINVAL
    assert f(BASE, BASE + 4096, 4, 2, None) == _capi.EINVAL          # unknown layout
    assert f(None, BASE + 4096, 4, 0, None) == _capi.EINVAL
    assert f(BASE + 4, BASE + 4096, 4, 0, None) == _capi.EINVAL      # not 16-byte aligned
    assert f(BASE, BASE + 16, 8, 0, None) == _capi.EOVERLAP          # out overlaps x
    # layout 1 writes 8 ceil(n/4) floats: for n = 5, out spans 64 bytes
    assert f(BASE + 48, BASE, 5, 1, None) == _capi.EOVERLAP
    rc = f(BASE, BASE + (1 << 44), (1 << 31) * 512, 0, None)
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()


def test_ablation_validation(L):
    v = L.sincos_f32_variant
    assert v(None, None, None, 0, 0, 0, 0, None) == _capi.OK
    assert v(BASE, BASE + 4096, BASE + 8192, 4, 2, 0, 0, None) == _capi.EINVAL    # CONTRACT
    assert v(BASE, BASE + 4096, BASE + 8192, 4, 0, 2, 0, None) == _capi.EINVAL    # method
    assert v(BASE, BASE + 4096, BASE + 8192, 4, 0, 0, 4, None) == _capi.EINVAL    # variant
    assert v(BASE + 4, BASE + 4100, BASE + 8196, 4, 0, 0, 0, None) == _capi.EINVAL  # 16-byte
    assert v(BASE, BASE + 8, BASE + 8192, 4, 0, 0, 0, None) == _capi.EOVERLAP
    d = L.sincos_f32_doublings
    F = ctypes.c_float * 16
    ss, cc = F(*([1.0] * 16)), F(*([-1.0] * 16))
    args = lambda **k: dict(dict(x=BASE, s=BASE + 4096, c=BASE + 8192, n=4, arith=0, nd=2, ss=ss,  # noqa: E731
                                 ns=4, cc=cc, nc=3, fix=1), **k)
    call = lambda a: d(a["x"], a["s"], a["c"], a["n"], a["arith"], a["nd"], a["ss"], a["ns"],  # noqa: E731
                       a["cc"], a["nc"], a["fix"], None)
    assert call(args(nd=9)) == _capi.EINVAL and "ndoub" in _capi.last_error()
    assert call(args(nd=-1)) == _capi.EINVAL
    assert call(args(ns=0)) == _capi.EINVAL and call(args(nc=17)) == _capi.EINVAL
    assert call(args(ss=None)) == _capi.EINVAL
    assert call(args(arith=2)) == _capi.EINVAL
    assert call(args(c=BASE + 4098)) == _capi.EINVAL
    assert call(args(n=0, ss=None)) == _capi.EINVAL      # coefficients are checked first


def test_fit_step_validation_and_workspace(L):
    wb = L.sinusoid_f32_fit_step_workspace_bytes
    assert wb(-1, 4) == -1 and wb(4, -1) == -1
    assert wb(0, 64) == 0
    assert wb(4_194_304, 64) == 2048 * (3 * 64 + 1) * 4     # partials + loss partial per 2048 samples
    assert wb(2049, 65) == 2 * (3 * 128 + 1) * 4
    f = L.sinusoid_f32_fit_step
    t, yo, A, w, p = BASE, BASE + 65536, BASE + 2 * 65536, BASE + 3 * 65536, BASE + 4 * 65536
    loss, gA, gw, gp, ws = (BASE + k * 65536 for k in range(5, 10))
    need = wb(16, 8)
    ok = dict(t=t, yo=yo, N=16, A=A, w=w, p=p, K=8, loss=loss, gA=gA, gw=gw, gp=gp, ws=ws, wsb=need)

    def call(**kw):
        a = dict(ok, **kw)
        return f(a["t"], a["yo"], a["N"], a["A"], a["w"], a["p"], a["K"], a["loss"], a["gA"],
                 a["gw"], a["gp"], a["ws"], a["wsb"], None)
    assert call(N=-1) == _capi.EINVAL
    assert call(loss=None) == _capi.EINVAL
    assert call(yo=None) == _capi.EINVAL
    assert call(wsb=need - 4) == _capi.EINVAL and "workspace" in _capi.last_error()
    assert call(gA=A) == _capi.EOVERLAP                  # gradient into a parameter
    assert call(loss=gw + 4) == _capi.EOVERLAP           # loss inside gw
    assert call(ws=yo) == _capi.EOVERLAP                 # workspace over y_obs
    assert call(gp=gp + 2) == _capi.EINVAL               # misaligned
    rc = f(t, yo, (1 << 31) * 2048 + 1, A, w, p, 8, loss, gA, gw, gp, ws, 1 << 40, None)
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()


def test_size_limits_keep_grids_below_the_dispatch_limit(L):
    """The dispatch packet counts work-items in 32 bits: entry points with one
    workgroup per fixed slice reject sizes whose grid * block would reach
    2^32; grid-stride kernels take sizes up to 2^36 (beyond device memory)."""
    rc = L.sincos_f32_interleaved(BASE, BASE + (1 << 44), (1 << 36) + 4, 0, None)
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()
    src = BASE + (1 << 20)
    rc = L.huygens_f32(BASE, BASE + 65536, (1 << 36) + 1, src, 4, 1.0, 100.0,
                       BASE + 2 * 65536, BASE + 3 * 65536, None)
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()
    rc = L.sincos_pair_ceiling_f32(BASE, BASE + (1 << 44), (0xFFFFFFFF // 256) * 256 + 1, 1, None)
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()
    n_over = (0xFFFFFFFF // 1024) * 2048 + 1        # one 1024-thread workgroup too many
    rc = L.sinusoid_f32_backward(BASE, BASE, n_over, BASE, BASE, BASE, 4, BASE, BASE, BASE, BASE,
                                 1 << 40, None)
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()
    t, yo, A, w, p = BASE, BASE + 65536, BASE + 2 * 65536, BASE + 3 * 65536, BASE + 4 * 65536
    loss, gA, gw, gp, ws = (BASE + k * 65536 for k in range(5, 10))
    rc = L.sinusoid_f32_fit_step(t, yo, n_over, A, w, p, 8, loss, gA, gw, gp, ws, 1 << 40, None)
    assert rc == _capi.EINVAL and "too large" in _capi.last_error()
