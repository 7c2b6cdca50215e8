"""Property tests of the C ABI's host logic (no GPU work): the ragged form's
aliasing rules against a brute-force check of every pair of arrays, and the
launch-shape tuning parser against Python's json module.  Addresses are fake
and never dereferenced: on a machine without a GPU a table that passes the
checks ends in SINCOS_ENODEV, so the outcome of validation is visible."""
import ctypes
import json
import random

import pytest
from hypothesis import example, given, settings, strategies as st

from paper_cs_0406049_amd import _capi, build as hipbuild


@pytest.fixture(scope="module")
def L():
    import torch
    if torch.cuda.is_available():
        pytest.skip("fake addresses must not reach a GPU; these checks run where there is none")
    if not hipbuild.is_built():
        hipbuild.build()
    return _capi.lib()


BASE = 1 << 32


def expected_overlap(segs, lens):
    """True when the table breaks the ragged rules: within a segment, s and c
    overlap or x overlaps s or c other than exactly; across the table, two
    outputs overlap, or an input overlaps an output other than its own
    segment's exact in-place output.  Empty segments take no part."""
    outs, ins = [], []
    for j, ((x, s, c), n) in enumerate(zip(segs, lens)):
        if n == 0:
            continue
        outs += [(s, s + 4 * n, j), (c, c + 4 * n, j)]
        ins.append((x, x + 4 * n, j))

    def hit(a, b):
        return a[0] < b[1] and b[0] < a[1]
    for i in range(len(outs)):
        for k in range(i + 1, len(outs)):
            if hit(outs[i], outs[k]):
                return True
    for xi in ins:
        for o in outs:
            if hit(xi, o) and not (o[2] == xi[2] and o[0] == xi[0]):
                return True
    return False


def random_table(rng):
    """Segments over a small address range, so that overlaps are common:
    starts on a 4-byte grid, lengths 0..6, some inputs in place."""
    count = rng.randint(1, 7)
    segs, lens = [], []
    for _ in range(count):
        n = rng.choice([0, 1, 2, 3, 4, 6])
        x = BASE + 4 * rng.randint(0, 60)
        s = BASE + 4 * rng.randint(0, 60)
        c = BASE + 4 * rng.randint(0, 60)
        r = rng.random()
        if r < 0.15:
            s = x
        elif r < 0.3:
            c = x
        elif r < 0.6:   # outputs well apart from everything else
            s = BASE + 4096 + 256 * len(segs)
            c = BASE + 8192 + 256 * len(segs)
        segs.append((x, s, c))
        lens.append(n)
    return segs, lens


def test_ragged_aliasing_matches_brute_force(L):
    rng = random.Random(12345)
    seen = {True: 0, False: 0}
    for trial in range(4000):
        segs, lens = random_table(rng)
        S = (_capi.Seg * len(segs))(*[_capi.Seg(*t) for t in segs])
        N = (ctypes.c_int64 * len(lens))(*lens)
        want = expected_overlap(segs, lens)
        rc = L.sincos_f32_ragged(S, N, len(segs), None)
        if want:
            assert rc == _capi.EOVERLAP, (trial, segs, lens, _capi.last_error())
        else:
            assert rc in (_capi.ENODEV, _capi.OK), (trial, segs, lens, rc, _capi.last_error())
            assert rc == _capi.OK or all(n == 0 for n in lens) or "device" in _capi.last_error()
        seen[want] += 1
    assert seen[True] > 500 and seen[False] > 500, seen   # both outcomes well covered


# --- tuning parser -------------------------------------------------------

BUILTIN = {"plain": {"block": 64, "unroll": 1, "grid": 0, "lds": 7168},
           "ragged": {"block": 256, "unroll": 1, "grid": 0, "lds": 0}}

field = st.sampled_from(["block", "unroll", "grid", "lds"])
value = st.one_of(st.sampled_from([0, 1, 2, 4, 8, 64, 128, 192, 256, 512, 1024, 1088, 3, 65,
                                   65536, 65537]),
                  st.integers(-5, 2000), st.integers(-(1 << 40), 1 << 40))
shape = st.dictionaries(field, value, max_size=4)
document = st.dictionaries(st.sampled_from(["plain", "ragged"]), shape, max_size=2)


def valid_shape(sh):
    return (64 <= sh["block"] <= 1024 and sh["block"] % 64 == 0 and sh["unroll"] in (1, 2, 4, 8)
            and sh["grid"] >= 0 and 0 <= sh["lds"] <= 65536)


@settings(max_examples=400, deadline=None)
@given(doc=document, indent=st.sampled_from([None, 0, 2]))
def test_tuning_accepts_exactly_the_valid_documents(L, doc, indent):
    """A well-formed document is accepted exactly when every shape it sets
    (over the built-in defaults) is valid, and then read back as set; a
    rejected one leaves the shapes in effect unchanged."""
    _capi.set_tuning(None)
    before = _capi.get_tuning()
    want = {f: dict(BUILTIN[f], **doc.get(f, {})) for f in BUILTIN}
    in_int = all(-(1 << 31) <= v <= (1 << 31) - 1 for sh in doc.values() for v in sh.values())
    ok = in_int and all(valid_shape(want[f]) for f in want)
    rc = L.sincos_set_tuning(json.dumps(doc, indent=indent).encode())
    try:
        if ok:
            assert rc == _capi.OK, (doc, _capi.last_error())
            assert _capi.get_tuning() == want
        else:
            assert rc == _capi.EINVAL, doc
            assert _capi.get_tuning() == before
    finally:
        _capi.set_tuning(None)


@settings(max_examples=600, deadline=None)
@example(text='{"plain": {"block": 0128}}')
@example(text='{"plain": {"grid": 00}}')
@example(text='\x0c{}')
@example(text='{"ragged": {}}\x0b')
@example(text='{"plain": {"grid": -0}}')
@example(text='{"plain": {"block": 1e2}}')
@example(text='{"ragged": {"block": 128}, "ragged": {"grid": 1}}')
@example(text='{"plain": {"block": 128, "block": 64}}')
@given(text=st.text(alphabet='{}[]:,"-. 0123456789eE\t\x0b\x0cplainraggedblockunrollgridldsx\\',
                    max_size=80))
def test_tuning_parser_never_accepts_what_json_rejects(L, text):
    """Arbitrary text: the call returns OK or EINVAL and never crashes; it is
    accepted only when json.loads reads the same document (the parser takes
    a subset of JSON), and a rejection changes nothing."""
    _capi.set_tuning(None)
    rc = L.sincos_set_tuning(text.encode())
    try:
        assert rc in (_capi.OK, _capi.EINVAL)
        if rc == _capi.OK:
            doc = json.loads(text)
            assert isinstance(doc, dict) and set(doc) <= {"plain", "ragged"}
            want = {f: dict(BUILTIN[f], **doc.get(f, {})) for f in BUILTIN}
            assert _capi.get_tuning() == want
        else:
            assert _capi.get_tuning() == BUILTIN
    finally:
        _capi.set_tuning(None)
