"""Pins of the oracle's adjoint and sinusoid-model functions against closed
forms and double-precision central differences of the exact model."""
import math

import numpy as np

FUSED, SPLIT = 0, 1


def test_pair_adjoint_closed_form(orc):
    rng = np.random.default_rng(1)
    x = rng.uniform(-10, 10, 5000)
    s = np.sin(x).astype(np.float32)
    c = np.cos(x).astype(np.float32)
    gs = rng.standard_normal(5000).astype(np.float32)
    gc = rng.standard_normal(5000).astype(np.float32)
    # one gradient present: the other term is exactly absent
    assert np.array_equal(orc.sincos_backward(s, c, np.ones_like(s), None), c)
    neg = orc.sincos_backward(s, c, None, np.ones_like(s))
    assert np.array_equal(neg, (np.float32(0) - s).astype(np.float32))
    assert np.all(orc.sincos_backward(s, c, None, None) == 0)
    # each product and the difference rounded once: |error| <= 2u (|gs c| + |gc s|)
    gx = orc.sincos_backward(s, c, gs, gc).astype(np.float64)
    exact = gs.astype(np.float64) * c - gc.astype(np.float64) * s
    scale = np.abs(gs.astype(np.float64) * c) + np.abs(gc.astype(np.float64) * s)
    assert np.all(np.abs(gx - exact) <= 2.01 * 2.0 ** -24 * scale + 1e-45)
    # chain rule: d/dx (gs sin x + gc cos x), central differences in double
    h = 1e-6
    fd = (gs * np.sin(x + h) + gc * np.cos(x + h) - gs * np.sin(x - h) - gc * np.cos(x - h)) / (2 * h)
    assert np.all(np.abs(gx - fd) <= 1e-6 * (np.abs(gs) + np.abs(gc)) + 1e-7)


def _model64(t, A, w, phi):
    return np.sin(np.outer(t, w) + phi) @ A


def _loss64(t, y, A, w, phi):
    r = _model64(t, A, w, phi) - y
    return 0.5 * float(r @ r)


def theta32(t, w, phi):
    """theta_ik = fl32(w_k t_i + phi_k) with one rounding (exact evaluation)."""
    from oracle import exact_binary32 as ex
    out = np.empty((t.size, w.size), np.float32)
    for k in range(w.size):
        wk, pk = ex.F32.from_float(float(w[k])), ex.F32.from_float(float(phi[k]))
        for i, ti in enumerate(t):
            out[i, k] = ex.fma(wk, ex.F32.from_float(float(ti)), pk).to_float()
    return out


def _small_problem(seed=3, N=300, K=4):
    rng = np.random.default_rng(seed)
    t = rng.uniform(0, 10, N).astype(np.float32)
    A = np.array([2.5, -0.7, 1.9, -3.1][:K], np.float32)
    w = rng.uniform(0.1, 3, K).astype(np.float32)
    phi = rng.uniform(-math.pi, math.pi, K).astype(np.float32)
    y = (_model64(t, A * 1.01, w * 1.001, phi + 0.01) + 0.01 * rng.standard_normal(N)).astype(np.float32)
    return t, A, w, phi, y


def test_sinusoid_forward_against_exact_model(orc):
    """y from binary32 theta and the method's pairs, against the double model
    on the same binary32 theta: within sum_k |A_k| (E_pair(theta) + K u) where
    E_pair is the pair's error bound at that angle."""
    t, A, w, phi, _ = _small_problem(N=4000)
    y = orc.sinusoid_forward(t, A, w, phi).astype(np.float64)
    theta = theta32(t, w, phi)
    ref = np.sin(theta.astype(np.float64)) @ A.astype(np.float64)
    k32 = 1.0 / (2 * math.pi)
    e_pair = 4.95e-7 + np.abs(theta.astype(np.float64)) * 4.1e-8 + \
        math.pi * np.abs(theta).astype(np.float64) * k32 * 2.0 ** -23
    bound = (e_pair * np.abs(A)).sum(1) + A.size * 2.0 ** -24 * np.abs(A).sum() * 1.01
    assert np.all(np.abs(y - ref) <= bound)


def test_sinusoid_adjoint_against_central_differences(orc):
    """The adjoint formulas (gA = sum g s, gphi = A sum g c, gw = A sum g c t)
    agree with double-precision central differences of the exact loss.  A
    dropped A_k or t_i factor or a sign error is off by O(1)."""
    t, A, w, phi, y = _small_problem()
    yf = orc.sinusoid_forward(t, A, w, phi)
    g = (yf - y).astype(np.float32)
    adj = orc.sinusoid_adjoint(t, g, A, w, phi)
    A64, w64, p64 = A.astype(np.float64), w.astype(np.float64), phi.astype(np.float64)
    t64, y64 = t.astype(np.float64), y.astype(np.float64)
    for name, key, base in (("A", "gA", A64), ("w", "gw", w64), ("phi", "gphi", p64)):
        for k in range(A.size):
            h = 1e-6 * max(1.0, abs(base[k]))
            plus, minus = base.copy(), base.copy()
            plus[k] += h
            minus[k] -= h
            args_p = {"A": A64, "w": w64, "phi": p64}
            args_m = dict(args_p)
            args_p[name] = plus
            args_m[name] = minus
            fd = (_loss64(t64, y64, args_p["A"], args_p["w"], args_p["phi"])
                  - _loss64(t64, y64, args_m["A"], args_m["w"], args_m["phi"])) / (2 * h)
            scale = adj["abs_" + ("phi" if name == "phi" else name)][k]
            assert abs(adj[key][k] - fd) <= 2e-4 * scale + 1e-6, (name, k, adj[key][k], fd)


def test_sinusoid_adjoint_abs_sums(orc):
    """With g = 1 the adjoint sums are plain column sums of the pairs."""
    t, A, w, phi, y = _small_problem(N=50)
    g = np.ones_like(t)
    adj = orc.sinusoid_adjoint(t, g, A, w, phi)
    s, c = orc.sincos(theta32(t, w, phi).ravel())
    s = s.reshape(t.size, A.size).astype(np.float64)
    c = c.reshape(t.size, A.size).astype(np.float64)
    assert np.allclose(adj["gA"], s.sum(0), rtol=0, atol=1e-12)
    assert np.allclose(adj["abs_A"], np.abs(s).sum(0), rtol=0, atol=1e-12)
    assert np.allclose(adj["gphi"], A * c.sum(0), rtol=0, atol=1e-12)
    assert np.allclose(adj["gw"], A * (c * t[:, None]).sum(0), rtol=0, atol=1e-9)
    # the forward's pairs are the same: y = sum_k A_k s_k accumulated by fma
    y32 = orc.sinusoid_forward(t, A, w, phi)
    assert np.allclose(y32, s @ A.astype(np.float64), rtol=0, atol=1e-5)
