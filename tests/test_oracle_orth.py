"""Pins of the oracle's Orth(.) against classical Gram-Schmidt (CPU only)."""
import numpy as np

import synth
from oracle.orth import orth, gram


def _gram_schmidt(X, h):
    """Classical Gram-Schmidt with one re-orthogonalisation pass, in a loop."""
    N = X.shape[0]
    V = X.reshape(N, -1).astype(np.float64).copy()
    W = np.zeros_like(V)
    R = np.zeros((N, N))
    for j in range(N):
        v = V[j].copy()
        for _ in range(2):
            for i in range(j):
                c = h ** 3 * np.dot(W[i], v)
                R[i, j] += c
                v -= c * W[i]
        R[j, j] = np.sqrt(h ** 3 * np.dot(v, v))
        W[j] = v / R[j, j]
    return W.reshape(X.shape), R


def test_orth_matches_gram_schmidt_and_properties():
    cfg = synth.custom("t", 9, 5.0, 1, 1.0, 0.5, 5)
    X = synth.orbitals(cfg)
    h = cfg.h
    W, R = orth(X, h)
    W2, R2 = _gram_schmidt(X, h)
    assert np.max(np.abs(W - W2)) < 1e-12 * np.max(np.abs(W))
    assert np.max(np.abs(R - R2)) < 1e-11 * np.max(np.abs(R))
    assert np.max(np.abs(gram(W, h) - np.eye(5))) < 1e-13
    assert np.all(np.diag(R) > 0) and np.allclose(np.tril(R, -1), 0)
    # X = W R  (orbital block times the triangular factor)
    Xr = np.einsum("ij,i...->j...", R, W)
    assert np.max(np.abs(Xr - X)) < 1e-11 * np.max(np.abs(X))


def test_orth_of_orthonormal_block_is_identity_map():
    cfg = synth.custom("t", 8, 4.0, 1, 1.0, 0.5, 3)
    W0, _ = orth(synth.orbitals(cfg), cfg.h)
    W1, R1 = orth(W0, cfg.h)
    assert np.max(np.abs(W1 - W0)) < 1e-13 * np.max(np.abs(W0))
    assert np.max(np.abs(R1 - np.eye(3))) < 1e-13
