"""Least-squares series for the general-doubling ablation (analysis only).

Sec. II's first method fits sin and cos of the quarter angle directly by
least squares.  For the ablation over the number of doublings n the same kind
of fit is redone for the angle 2 pi q / 2^n, q in [0, 1/2] (the reduced turn;
negative q follow by symmetry):
    sin(2 pi q / 2^n)     ~ q (ss[0] + ss[1] q^2 + ... + ss[ns-1] q^(2 ns - 2))
    cos(2 pi q / 2^n) - 1 ~ q^2 (cc[0] + cc[1] q^2 + ... + cc[nc-1] q^(2 nc - 2))
Reading: the paper names neither the sample set nor a weight; here the fit is
unweighted over uniformly spaced q, solved in double precision, and each
coefficient is then rounded to binary32 once.  The coefficients of the paper
itself are not the output of this fit to the last digit (they are typed in the
oracle from the printed decimals); the fit is only used to build series for
doubling counts the paper does not print.
"""
from __future__ import annotations

import numpy as np


def fit_series(ndoub: int, ns: int, nc: int, samples: int = 200001):
    """Binary32 (ss, cc) for n = ndoub doublings, ns sine and nc cosine terms."""
    if not (0 <= ndoub <= 16 and 1 <= ns <= 16 and 1 <= nc <= 16):
        raise ValueError("ndoub in [0, 16], ns and nc in [1, 16]")
    q = np.linspace(0.0, 0.5, samples)
    theta = 2.0 * np.pi * q / 2.0 ** ndoub
    # scale the variable to [0, 1] for conditioning, then undo the scaling
    z = 2.0 * q
    As = np.stack([z ** (2 * k + 1) for k in range(ns)], axis=1)
    a, *_ = np.linalg.lstsq(As, np.sin(theta), rcond=None)
    Ac = np.stack([z ** (2 * k + 2) for k in range(nc)], axis=1)
    b, *_ = np.linalg.lstsq(Ac, np.cos(theta) - 1.0, rcond=None)
    ss = np.array([a[k] * 2.0 ** (2 * k + 1) for k in range(ns)])
    cc = np.array([b[k] * 2.0 ** (2 * k + 2) for k in range(nc)])
    return ss.astype(np.float32), cc.astype(np.float32)


def fit_residual(ndoub: int, ss, cc, samples: int = 200001):
    """Largest |series - function| over q in [0, 1/2] for sine and cosine,
    evaluated in double with the binary32 coefficients."""
    q = np.linspace(0.0, 0.5, samples)
    theta = 2.0 * np.pi * q / 2.0 ** ndoub
    q2 = q * q
    ps = np.zeros_like(q)
    for k in reversed(range(len(ss))):
        ps = ps * q2 + float(ss[k])
    pc = np.zeros_like(q)
    for k in reversed(range(len(cc))):
        pc = pc * q2 + float(cc[k])
    return (float(np.max(np.abs(q * ps - np.sin(theta)))),
            float(np.max(np.abs(1.0 + q2 * pc - np.cos(theta)))))
