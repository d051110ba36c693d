"""Orth(.) of Algorithm B step 5 (oracle, FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Orth(X) is the unique W = X R^-1 with R upper triangular, diag(R) > 0 and
<W^T W> = I in the grid inner product <a, b> = h^3 sum a b.  Section 3.2
orthonormalises through QR (the OptM-QR description) and computes that QR
through a Cholesky factorisation of the Gram matrix; a Cholesky factor has a
positive diagonal, so the factor is exactly this unique one.  The oracle
computes it with Householder QR (numpy.linalg.qr) and fixes the signs, which
is independent of any Cholesky-based route and equal to it in exact
arithmetic.

Parity: pinned against classical Gram-Schmidt written out in a loop
(tests/test_oracle_orth.py) and against the defining properties.
"""
from __future__ import annotations

import numpy as np


def orth(X, h):
    """Return (W, R) with X = W R (as blocks of orbitals), R upper, diag R > 0."""
    N = X.shape[0]
    shape = X.shape
    A = np.sqrt(h ** 3) * X.reshape(N, -1).T          # Ng x N, columns = orbitals
    Q, R = np.linalg.qr(A, mode="reduced")
    sgn = np.sign(np.diag(R))
    sgn[sgn == 0] = 1.0
    Q = Q * sgn[None, :]
    R = R * sgn[:, None]
    W = (Q.T / np.sqrt(h ** 3)).reshape(shape)
    return W, R


def gram(X, h):
    """<X^T X> = h^3 X X^T as an N x N matrix."""
    N = X.shape[0]
    Xf = X.reshape(N, -1)
    return h ** 3 * (Xf @ Xf.T)
