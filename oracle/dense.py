"""Brute-force dense linear algebra on tiny grids (oracle, FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Used to pin the minimisation: the minimiser of the constrained problem
(section 2.1, eq. "emin") satisfies the Kohn-Sham equation H(rho) U = U Lambda
(section 2.2); for a linear Hamiltonian the minimum is sum_i f_i lambda_i over
the N lowest eigenvalues, and for the full nonlinear model a converged
self-consistent-field solve with dense diagonalisation reaches the same
minimiser on a gapped instance.

Parity: scipy.linalg.eigh is the library routine; the dense matrix is built
column by column from the oracle's own operator (ks.kinetic).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from . import ks


def kinetic_matrix(n, h):
    """Dense K = -1/2 Delta_h, Ng x Ng, by applying K to each unit vector."""
    ng = n ** 3
    E = np.eye(ng).reshape(ng, n, n, n)
    return ks.kinetic(E, h).reshape(ng, ng).T


def nonlocal_matrix(sys: ks.System):
    """Dense V_nloc (section 2.1), Ng x Ng: (V u)_g = sum_l xi_l(g) h^3 sum_g'
    xi_l(g') u_g', i.e. the matrix h^3 Xi^T Xi of the projector rows."""
    Xi = ks.projectors(sys).reshape(-1, sys.n ** 3)
    return sys.h ** 3 * (Xi.T @ Xi)


def lowest_eigs(Hmat, k):
    w, v = scipy.linalg.eigh(Hmat, subset_by_index=[0, k])
    return w, v


def linear_minimum(sys: ks.System, vext=None):
    """min E for the linear problem (terms KIN | EXT): sum f_i lambda_i."""
    n, h = sys.n, sys.h
    if vext is None:
        vext = ks.external_potential(sys)
    H = kinetic_matrix(n, h)
    if sys.terms & ks.TERM_EXT:
        H = H + np.diag(vext.reshape(-1))
    if ks.nonlocal_active(sys):
        H = H + nonlocal_matrix(sys)
    N = sys.norb
    w, _ = lowest_eigs(H, N)
    return float(np.sum(sys.occ * w[:N])), w


def scf(sys: ks.System, mix=0.3, tol=1e-12, maxit=2000, vext=None):
    """Dense SCF: fill the N lowest eigenvectors of H(rho), linear density mixing.

    Returns (energy terms, orbitals [N, n, n, n], eigenvalues, gap).
    """
    n, h = sys.n, sys.h
    N = sys.norb
    if vext is None:
        vext = ks.external_potential(sys)
    K = kinetic_matrix(n, h)
    rho = np.full((n, n, n), np.sum(sys.occ) / sys.L ** 3)
    for it in range(maxit):
        VH = ks.poisson(rho, h)
        _, vx = ks.exchange(rho, h)
        veff = vext + VH + vx
        H = K + np.diag(veff.reshape(-1))
        w, v = lowest_eigs(H, N)
        U = (v[:, :N].T / np.sqrt(h ** 3)).reshape(N, n, n, n)
        rho_new = ks.density(U, sys.occ)
        err = float(np.max(np.abs(rho_new - rho)))
        rho = (1.0 - mix) * rho + mix * rho_new
        if err < tol:
            break
    terms = ks.energy(U, sys, vext)
    return terms, U, w, float(w[N] - w[N - 1]), it
