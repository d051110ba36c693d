"""Plain conjugate gradients for the periodic Poisson problem (oracle, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Solves -Delta_h V = 4 pi (f - mean f) for the zero-mean V by textbook CG
(Hestenes-Stiefel), written independently of the FFT solve in ks.poisson so
that each pins the other.  The operator is applied through ks.laplacian.
"""
from __future__ import annotations

import numpy as np

from . import ks


def poisson_cg(f, h, rtol=1e-13, maxit=20000):
    b = 4.0 * np.pi * (f - np.mean(f))
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = float(np.sum(r * r))
    bnorm = np.sqrt(float(np.sum(b * b)))
    it = 0
    while it < maxit and np.sqrt(rr) > rtol * bnorm:
        Ap = -ks.laplacian(p, h)
        alpha = rr / float(np.sum(p * Ap))
        x += alpha * p
        r -= alpha * Ap
        rr_new = float(np.sum(r * r))
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
    return x - np.mean(x), it
