"""Seeded synthetic inputs for every workload of this package.

This module holds input generation only: random angles, lengths, sample
times, parameters, arrival times, and the series coefficients given to the
general-doubling ablation.  It contains none of the sine-cosine
method's arithmetic, so both the GPU path and the CPU oracle can consume what
it makes without sharing any of the method's code.

All draws use ``numpy.random.default_rng(seed)``; uniform draws are made in
binary64 and then rounded to binary32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

# ---------------------------------------------------------------------------
# Plain method


def plain_small(n: int = 1 << 20, seed: int = 0) -> np.ndarray:
    """1,048,576 angles i.i.d. uniform in [-8 pi, 8 pi)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-8.0 * math.pi, 8.0 * math.pi, n).astype(np.float32)


def plain_roofline(n: int = 1 << 28, seed: int = 1) -> np.ndarray:
    """268,435,456 angles: half uniform in [-pi, pi), half uniform in
    [-1e4, 1e4), then shuffled (one array of 1 GiB)."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, np.float32)
    h = n // 2
    out[:h] = rng.uniform(-math.pi, math.pi, h)
    out[h:] = rng.uniform(-1e4, 1e4, n - h)
    rng.shuffle(out)
    return out


def uniform_angles(n: int, lo: float, hi: float, seed: int) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, n).astype(np.float32)


# ---------------------------------------------------------------------------
# Ragged batch


def ragged_lengths(count: int = 4096, lo: float = 100.0, hi: float = 1e6, seed: int = 2):
    """Lengths floor(10^U(log10 lo, log10 hi)): log-uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(math.log10(lo), math.log10(hi), count)
    return np.floor(10.0 ** e).astype(np.int64)


def ragged_batch(count: int = 4096, seed: int = 2, lo: float = 100.0, hi: float = 1e6):
    """(lengths, list of angle arrays): angles uniform in [-100 pi, 100 pi)."""
    lens = ragged_lengths(count, lo, hi, seed)
    rng = np.random.default_rng(seed + 1000)
    flat = rng.uniform(-100.0 * math.pi, 100.0 * math.pi, int(lens.sum())).astype(np.float32)
    offs = np.concatenate([[0], np.cumsum(lens)])
    return lens, [flat[offs[i]:offs[i + 1]] for i in range(count)]


# ---------------------------------------------------------------------------
# Sinusoid-model fitting


@dataclass
class SinusoidProblem:
    t: np.ndarray      # [N] sample times
    A: np.ndarray      # [K] amplitudes
    w: np.ndarray      # [K] angular frequencies
    phi: np.ndarray    # [K] phases
    y_obs: np.ndarray  # [N] observations
    A_true: np.ndarray
    w_true: np.ndarray
    phi_true: np.ndarray


def sinusoid_problem(N: int = 4_194_304, K: int = 64, seed: int = 3,
                     t_max: float = 1000.0, noise: float = 0.01,
                     chunk: int = 1 << 16) -> SinusoidProblem:
    """Model y(t) = sum_k A_k sin(w_k t + phi_k).

    One rng stream, drawn in this order: t ~ U[0, t_max] (N), A ~ N(0, 1),
    w ~ U[0.1, 10], phi ~ U[-pi, pi) (K each); the observations come from
    perturbed parameters A' = A + 0.01 N(0,1), phi' = phi + 0.01 N(0,1),
    w' = w (1 + 1e-5 N(0,1)), evaluated in binary64 with the system sine, plus
    N(0, noise^2) noise.  The fit starts from (A, w, phi)."""
    rng = np.random.default_rng(seed)
    t = rng.uniform(0.0, t_max, N)
    A = rng.standard_normal(K)
    w = rng.uniform(0.1, 10.0, K)
    phi = rng.uniform(-math.pi, math.pi, K)
    A_t = A + 0.01 * rng.standard_normal(K)
    phi_t = phi + 0.01 * rng.standard_normal(K)
    w_t = w * (1.0 + 1e-5 * rng.standard_normal(K))
    y = np.empty(N, np.float64)
    for lo in range(0, N, chunk):
        hi = min(N, lo + chunk)
        y[lo:hi] = np.sin(np.outer(t[lo:hi], w_t) + phi_t) @ A_t
    y += noise * rng.standard_normal(N)
    f = lambda a: np.ascontiguousarray(a, dtype=np.float32)  # noqa: E731
    return SinusoidProblem(f(t), f(A), f(w), f(phi), f(y), f(A_t), f(w_t), f(phi_t))


# ---------------------------------------------------------------------------
# Served requests


@dataclass
class RequestStream:
    sizes: np.ndarray        # [R] elements per request
    unit_gaps: np.ndarray    # [R] Exp(1) inter-arrival draws; divide by the rate
    offsets: np.ndarray      # [R] start of each request's window in the angle pool
    pool: np.ndarray         # angle pool, uniform in [-1e3, 1e3)


def request_stream(count: int = 10_000, lo: float = 1e3, hi: float = 1e7, seed: int = 4,
                   pool_elems: int = 1 << 26) -> RequestStream:
    """Requests of log-uniform size in [lo, hi]; Poisson arrivals (unit-rate
    exponential gaps); each request's angles are a window of a shared pool of
    angles uniform in [-1e3, 1e3) (the pool is resident on the device)."""
    rng = np.random.default_rng(seed)
    e = rng.uniform(math.log10(lo), math.log10(hi), count)
    sizes = np.floor(10.0 ** e).astype(np.int64)
    gaps = rng.exponential(1.0, count)
    pool_elems = max(pool_elems, int(sizes.max()))
    # window starts are multiples of 64 elements (256 B) so device pointers stay aligned
    slots = (pool_elems - sizes) // 64
    offsets = (rng.integers(0, np.maximum(slots, 0) + 1) * 64).astype(np.int64)
    pool = rng.uniform(-1e3, 1e3, pool_elems).astype(np.float32)
    return RequestStream(sizes, gaps, offsets, pool)


# ---------------------------------------------------------------------------
# Series for the general-doubling ablation


def taylor_series(ndoub: int, ns: int, nc: int):
    """Binary32 Taylor coefficients of sin and cos of a q, a = 2 pi / 2^ndoub,
    in the form the general-doubling ablation takes: s1 = q (ss[0] + ss[1] q^2
    + ...), c1 = 1 + q^2 (cc[0] + cc[1] q^2 + ...).  Any coefficients serve
    for timing and for comparing two implementations bit for bit."""
    a = 2.0 * math.pi / 2.0 ** ndoub
    ss = [(-1) ** k * a ** (2 * k + 1) / math.factorial(2 * k + 1) for k in range(ns)]
    cc = [(-1) ** (k + 1) * a ** (2 * k + 2) / math.factorial(2 * k + 2) for k in range(nc)]
    return np.array(ss).astype(np.float32), np.array(cc).astype(np.float32)


# ---------------------------------------------------------------------------
# Huygens diffraction (the author's application)


@dataclass
class HuygensProblem:
    xo: np.ndarray    # [P] screen x (wavelengths)
    yo: np.ndarray    # [P] screen y
    src: np.ndarray   # [S, 4] source x, y, amplitude, phase
    k: float          # wavenumber (2 pi: lengths in wavelengths)
    L: float          # aperture-to-screen distance


def huygens_problem(screen_side: int = 512, aperture_side: int = 64, seed: int = 5,
                    D: float = 256.0, W: float = 256.0, L: float = 2.0e4,
                    aberration: float = 0.1, lens: bool = True) -> HuygensProblem:
    """A square aperture of side D sampled by aperture_side^2 point sources on a
    regular grid, with seeded apodization a ~ U[0.5, 1]/S; phases of a thin lens
    focusing on the screen centre (if lens) plus seeded aberration N(0, aberration^2);
    a square screen of side W, screen_side^2 points, at distance L.  Lengths in
    wavelengths (k = 2 pi).  The phases are made in binary64, then rounded."""
    rng = np.random.default_rng(seed)
    k = 2.0 * math.pi
    g = (np.arange(aperture_side) + 0.5) / aperture_side * D - D / 2
    xa, ya = np.meshgrid(g, g, indexing="xy")
    xa, ya = xa.ravel(), ya.ravel()
    S = xa.size
    a = rng.uniform(0.5, 1.0, S) / S
    phi = np.zeros(S)
    if lens:
        phi -= k * (np.sqrt(xa * xa + ya * ya + L * L) - L)
    phi += aberration * rng.standard_normal(S)
    src = np.stack([xa, ya, a, phi], axis=1).astype(np.float32)
    h = (np.arange(screen_side) + 0.5) / screen_side * W - W / 2
    xo, yo = np.meshgrid(h, h, indexing="xy")
    return HuygensProblem(xo.ravel().astype(np.float32), yo.ravel().astype(np.float32),
                          np.ascontiguousarray(src), k, L)
