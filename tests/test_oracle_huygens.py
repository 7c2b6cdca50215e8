"""Pins of the oracle's Huygens point-source sum: a single source in closed
form, the exact double-precision model within a derived bound, the
Fraunhofer (far-field) limit of a square aperture, symmetry, and the block
structure of the sum (four contiguous blocks of sources, each summed in
order, added in block order) against the plain sum of each block."""
import math

import numpy as np
import pytest

import oracle

U = 2.0 ** -24
K = 2.0 * math.pi


def exact_field(xo, yo, src, k, L):
    """U_i = sum_j a_j / r exp(i (k (r - L) + phi_j)) in double precision on the
    same binary32 inputs."""
    xo = xo.astype(np.float64)[:, None]
    yo = yo.astype(np.float64)[:, None]
    xa, ya, a, phi = (src[:, i].astype(np.float64)[None, :] for i in range(4))
    rho2 = (xo - xa) ** 2 + (yo - ya) ** 2
    r = np.sqrt(rho2 + float(L) ** 2)
    d = rho2 / (r + float(L))
    theta = float(np.float32(k)) * d + phi
    w = a / r
    return (w * np.cos(theta)).sum(1), (w * np.sin(theta)).sum(1), w, theta, d


def field_bound(w, theta, d, k, blocks=oracle.HUYGENS_BLOCKS):
    """Per-point bound on |U32 - U64|: each term's pair error E_pair(theta)
    plus its phase error, the error of its weight, and the sum: a recursive
    fma sum over each block of ceil(S / blocks) terms, then blocks - 1
    additions.  Relative errors to first order in U: rho^2 <= 4U (dx, dy,
    dy^2, the fma); r <= 3U (the sum with L^2, the square root); e = r + L
    <= 4U.  With g = 1/(r e) the same rounded r enters the numerator and the
    denominator of d = rho^2 (r g) and cancels: d = rho^2 / e times four
    roundings, <= 4U + 4U + 4U = 12U (14U used); theta adds one rounding of
    itself.  w = a (e g) = a / r times four roundings, <= 3U + 4U = 7U (8U
    used).  Where r e is not a normal binary32 the term divides twice
    instead: d <= 4U + 4U + U = 9U, w <= 3U + U = 4U, inside the same bound."""
    x1 = np.abs(theta) / (2 * math.pi)
    e_pair = 4.95e-7 + np.abs(theta) * 4.1e-8 + math.pi * np.maximum(x1, 1e-30) * 2 * U
    e_phase = abs(k) * 14 * U * d + 2 * U * np.abs(theta)
    S = w.shape[1]
    per = -(-S // blocks)
    return (w * (e_pair + e_phase + 8 * U)).sum(1) + 2 * (per + blocks) * U * w.sum(1)


def test_single_source_closed_form(orc):
    xo = np.array([0.0, 3.0, -7.5, 20.0], np.float32)
    yo = np.array([0.0, 4.0, 2.25, -9.0], np.float32)
    src = np.array([[1.0, -2.0, 0.75, 0.3]], np.float32)
    L = 1000.0
    re, im = orc.huygens(xo, yo, src, K, L)
    er, ei, w, th, d = exact_field(xo, yo, src, K, L)
    b = field_bound(w, th, d, K)
    assert np.all(np.hypot(re - er, im - ei) <= b)
    # on the source's axis the path difference is 0: U = a/L e^{i phi}
    re0, im0 = orc.huygens(np.array([1.0], np.float32), np.array([-2.0], np.float32), src, K, L)
    assert abs(re0[0] - 0.75 / L * math.cos(0.3)) < 2e-7 * 0.75 / L * 10
    assert abs(im0[0] - 0.75 / L * math.sin(0.3)) < 2e-7 * 0.75 / L * 10


@pytest.mark.parametrize("blocks", [1, 4])
def test_against_exact_model_within_bound(orc, blocks):
    rng = np.random.default_rng(6)
    S, P = 303, 500
    src = np.stack([rng.uniform(-50, 50, S), rng.uniform(-50, 50, S), rng.uniform(0, 1, S) / S,
                    rng.uniform(-3, 3, S)], 1).astype(np.float32)
    xo = rng.uniform(-200, 200, P).astype(np.float32)
    yo = rng.uniform(-200, 200, P).astype(np.float32)
    L = 5000.0
    re, im = orc.huygens(xo, yo, src, K, L, threads=4, blocks=blocks)
    er, ei, w, th, d = exact_field(xo, yo, src, K, L)
    err = np.hypot(re - er, im - ei)
    b = field_bound(w, th, d, K, blocks)
    assert np.all(err <= b), (err / b).max()
    # and the bound is not vacuous: the field itself is far larger
    assert np.median(b) < 1e-3 * np.median(np.hypot(er, ei)) * 10


# Geometries at the ends of the range, lengths scaled by s and k by 1/s (the
# field is scale-free), so that the phases stay moderate and the bound
# measures accuracy: r near 2^50 (one reciprocal; multiplying rho^2 by r
# before the reciprocal would overflow there), L = 2^-64 (r (r + L) below
# the normal range: two divisions) and L = 1.6e19 (r (r + L) above it).
EXTREME_CASES = {
    "big_r": (2.0 ** 44, 2.0 ** 45, 2.0 ** 50, 2.0 ** 44),
    "tiny_L": (2.0 ** -66, 2.0 ** -65, 2.0 ** -64, 2.0 ** -66),
    "huge_L": (2.0 ** 57, 2.0 ** 58, 1.6e19, 2.0 ** 57),
}


def extreme_case(name, S=57, P=64):
    """(xo, yo, src, k, L) for one of EXTREME_CASES: sources within +-src_half
    and points within +-pt_half, k = 2 pi / s."""
    src_half, pt_half, L, s = EXTREME_CASES[name]
    rng = np.random.default_rng(len(name))
    src = np.stack([rng.uniform(-1, 1, S) * src_half, rng.uniform(-1, 1, S) * src_half,
                    rng.uniform(0, 1, S) / S, rng.uniform(-3, 3, S)], 1).astype(np.float32)
    xo = (rng.uniform(-1, 1, P) * pt_half).astype(np.float32)
    yo = (rng.uniform(-1, 1, P) * pt_half).astype(np.float32)
    return xo, yo, src, float(np.float32(K / s)), L


def shared_fraction(xo, yo, src, L):
    """Fraction of terms for which r (r + L), formed in binary32 as the
    oracle forms it, is a normal binary32 (the one-reciprocal branch)."""
    f = np.float32
    dx = (xo[:, None] - src[None, :, 0]).astype(f)
    dy = (yo[:, None] - src[None, :, 1]).astype(f)
    rho2 = (dx.astype(np.float64) ** 2 + (dy * dy).astype(f)).astype(f)
    r = np.sqrt((rho2 + f(f(L) * f(L))).astype(f)).astype(f)
    e = (r + f(L)).astype(f)
    with np.errstate(over="ignore", under="ignore"):
        x = (r.astype(np.float64) * e).astype(f)
    return float(((x >= np.finfo(f).tiny) & (x <= np.finfo(f).max)).mean())


@pytest.mark.parametrize("name,shared", [("big_r", 1.0), ("tiny_L", 0.0), ("huge_L", 0.0)])
def test_extreme_geometries_within_bound(orc, name, shared):
    """At both ends of the range the field stays finite and within the bound
    of the exact model, in the branch the case is built for."""
    xo, yo, src, k, L = extreme_case(name)
    assert shared_fraction(xo, yo, src, L) == shared
    re, im = orc.huygens(xo, yo, src, k, L, threads=4)
    er, ei, w, th, d = exact_field(xo, yo, src, k, L)
    b = field_bound(w, th, d, k)
    err = np.hypot(re.astype(np.float64) - er, im.astype(np.float64) - ei)
    assert np.all(np.isfinite(re)) and np.all(np.isfinite(im))
    assert np.all(err <= b), (err / b).max()
    assert np.median(b) < 1e-2 * np.median(np.hypot(er, ei))


def block_combination(orc, xo, yo, src, k, L, blocks):
    """The blocked sum rebuilt from plain (one-block) sums of each block,
    added in block order in binary32."""
    S = src.shape[0]
    per = -(-S // blocks) if S else 0
    re = im = None
    for b in range(blocks):
        lo, hi = min(S, b * per), min(S, (b + 1) * per)
        br, bi = orc.huygens(xo, yo, src[lo:hi], k, L, blocks=1)
        re, im = (br, bi) if re is None else ((re + br).astype(np.float32),
                                             (im + bi).astype(np.float32))
    return re, im


@pytest.mark.parametrize("S", [0, 1, 3, 4, 5, 203, 1000])
def test_blocked_sum_is_the_block_order_sum_of_plain_sums(orc, S):
    """The default sum is four contiguous blocks of ceil(S/4) sources, each
    the plain sum in source order, added in block order: bit for bit."""
    rng = np.random.default_rng(S + 11)
    src = np.stack([rng.uniform(-50, 50, S), rng.uniform(-50, 50, S), rng.uniform(0, 1, S),
                    rng.uniform(-3, 3, S)], 1).astype(np.float32).reshape(S, 4)
    xo = rng.uniform(-200, 200, 400).astype(np.float32)
    yo = rng.uniform(-200, 200, 400).astype(np.float32)
    re, im = orc.huygens(xo, yo, src, K, 5000.0)
    wr, wi = block_combination(orc, xo, yo, src, K, 5000.0, orc.HUYGENS_BLOCKS)
    assert np.array_equal(re.view(np.uint32), wr.view(np.uint32))
    assert np.array_equal(im.view(np.uint32), wi.view(np.uint32))
    if S >= 203:
        # the block order is a real choice: the plain sum differs in the last bits
        pr, pi = orc.huygens(xo, yo, src, K, 5000.0, blocks=1)
        assert not np.array_equal(pr.view(np.uint32), re.view(np.uint32))


def test_fraunhofer_limit_of_a_square_aperture(orc):
    """Plane wave, M x M sources of pitch p, far screen: |U| = |D_M(u) D_M(v)| / L
    with D_M(u) = sin(M u/2) / (M sin(u/2)), u = k p x / L (the Dirichlet
    kernel, the sampled aperture's far-field pattern)."""
    M, p, L = 32, 1.0, 1.0e5
    g = (np.arange(M) - (M - 1) / 2) * p
    xa, ya = np.meshgrid(g, g)
    S = M * M
    src = np.stack([xa.ravel(), ya.ravel(), np.full(S, 1.0 / S), np.zeros(S)], 1).astype(np.float32)
    xs = np.array([0.0, 150.0, 400.0, 700.0, 1200.0, 2100.0], np.float32)
    xo = np.concatenate([xs, xs]).astype(np.float32)
    yo = np.concatenate([np.zeros_like(xs), xs]).astype(np.float32)
    re, im = orc.huygens(xo, yo, src, K, L, threads=4)
    amp = np.hypot(re, im) * L

    def dirichlet(u):
        u = np.asarray(u, np.float64)
        out = np.ones_like(u)
        nz = np.abs(np.sin(u / 2)) > 1e-12
        out[nz] = np.sin(M * u[nz] / 2) / (M * np.sin(u[nz] / 2))
        return np.abs(out)
    ux = K * p * xo.astype(np.float64) / L
    uy = K * p * yo.astype(np.float64) / L
    want = dirichlet(ux) * dirichlet(uy)
    assert abs(amp[0] - 1.0) < 1e-3                 # on axis: all sources in phase
    assert np.all(np.abs(amp - want) < 0.01), np.c_[amp, want]


def test_mirror_symmetry(orc):
    M = 16
    g = (np.arange(M) - (M - 1) / 2) * 3.0
    xa, ya = np.meshgrid(g, g)
    S = M * M
    src = np.stack([xa.ravel(), ya.ravel(), np.full(S, 1.0 / S), np.zeros(S)], 1).astype(np.float32)
    x = np.linspace(0, 300, 37).astype(np.float32)
    y = np.linspace(-100, 200, 37).astype(np.float32)
    L = 3000.0
    r1, i1 = orc.huygens(x, y, src, K, L)
    r2, i2 = orc.huygens(-x, y, src, K, L)
    r3, i3 = orc.huygens(y, x, src, K, L)
    tol = 64 * U * np.abs(src[:, 2]).sum() / L * 10
    assert np.all(np.hypot(r1 - r2, i1 - i2) < tol)
    assert np.all(np.hypot(r1 - r3, i1 - i3) < tol)


def test_no_sources_gives_zero(orc):
    re, im = orc.huygens(np.zeros(3, np.float32), np.zeros(3, np.float32),
                         np.zeros((0, 4), np.float32), K, 10.0)
    assert np.all(re == 0) and np.all(im == 0) and not np.any(np.signbit(re))
