"""Pins of the oracle's Algorithm M (CPU only).

The converged result of the inner loop is the minimiser of eq. "emin"; on
inputs where that minimiser is independently computable (closed-shell free
box, linear Hamiltonian, dense self-consistent field on a gapped instance)
the oracle must reach it.  Along a trajectory, every accepted step must meet
eq. "ene-de", C must not increase, and the invariants of section 2.2 and 3.2
must hold.
"""
import json
import os

import numpy as np
import pytest

import synth
from oracle import ks, algm, dense
from oracle.orth import gram

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_default_parameters_are_the_papers():
    c = json.load(open(os.path.join(GOLD, "paper_constants.json")))
    p = algm.Params()
    assert (p.rho1, p.delta, p.eta) == (c["rho1"], c["delta"], c["eta"])


def test_lambda_max_of_kinetic_operator_is_the_dense_maximum():
    n, h = 8, 0.6
    K = dense.kinetic_matrix(n, h)
    w = np.linalg.eigvalsh(K)
    assert abs(w[-1] - algm.lambda_max_kinetic(h)) < 1e-10 * w[-1]


@pytest.mark.parametrize("N", [1, 7])
def test_free_box_closed_shell_reaches_dense_minimum(N):
    n, L = 8, 5.0
    cfg = synth.custom("t", n, L, 0, 1.0, 0.5, N, seed_id=31)
    sys_ = ks.System(n, L, np.zeros((0, 3)), np.zeros(0), np.zeros(0),
                     synth.occupations(cfg), ks.TERM_KIN)
    w = np.linalg.eigvalsh(dense.kinetic_matrix(n, L / n))
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_)
    A.run(3000, tol=1e-15)
    assert abs(A.E - 2 * np.sum(w[:N])) < 1e-10


def test_linear_problem_reaches_dense_minimum():
    cfg = synth.custom("t", 10, 6.0, 2, (1.0, 2.0), (0.45, 0.7), 2, seed_id=5)
    R, Z, s = synth.atoms(cfg)
    sys_ = ks.System(10, 6.0, R, Z, s, synth.occupations(cfg), ks.TERM_KIN | ks.TERM_EXT)
    Emin, w = dense.linear_minimum(sys_)
    assert w[2] - w[1] > 1e-2
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_)
    A.run(3000, tol=1e-15)
    assert abs(A.E - Emin) < 1e-10


@pytest.mark.parametrize("n,L,M,N,seed", [(8, 5.0, 2, 1, 5), (10, 6.0, 3, 2, 7)])
def test_nonlinear_problem_reaches_dense_scf(n, L, M, N, seed):
    cfg = synth.custom("t", n, L, M, (1.0, 2.0), (0.45, 0.7), N, seed_id=seed)
    R, Z, s = synth.atoms(cfg)
    sys_ = ks.System(n, L, R, Z, s, synth.occupations(cfg))
    terms, _, _, gap, _ = dense.scf(sys_, mix=0.5)
    assert gap > 1e-2
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_)
    A.run(5000, tol=1e-16)
    assert abs(A.E - terms.E) < 1e-9


def _small16():
    cfg = synth.CONFIGS["small16"]
    R, Z, s = synth.atoms(cfg)
    return ks.System(cfg.n, cfg.L, R, Z, s, synth.occupations(cfg)), cfg


def test_trajectory_invariants_small16():
    sys_, cfg = _small16()
    p = algm.Params()
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_, p)
    C_prev = A.C
    for _ in range(50):
        Z = A.direction()
        # <z_i, w_i> = 0 for the diagonal-sigma direction (section 3.2)
        assert np.max(np.abs(ks.inner(Z, A.W, sys_.h))) < 1e-10
        rec = A.step()
        assert rec.accepted
        # eq. "ene-de" at the accepted tau, against the C before the update
        assert rec.E <= C_prev - p.rho1 * rec.tau * rec.zz + 1e-12
        assert rec.C <= C_prev + 1e-12
        C_prev = rec.C
        assert np.max(np.abs(gram(A.W, sys_.h) - np.eye(cfg.norb))) < 1e-12
        rho = ks.density(A.W, sys_.occ)
        assert abs(sys_.dv * rho.sum() - sys_.occ.sum()) < 1e-11


def test_monotone_decrease_with_eta_zero():
    sys_, cfg = _small16()
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_, algm.Params(eta=0.0))
    E_prev = A.E
    for _ in range(40):
        rec = A.step()
        assert rec.E < E_prev
        E_prev = rec.E


def test_backtracking_rejects_oversized_step():
    """A huge initial tau must be cut by delta until eq. "ene-de" holds."""
    sys_, cfg = _small16()
    p = algm.Params(tau_init=50.0)
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_, p)
    C0 = A.C
    rec = A.step()
    assert rec.s >= 1 and rec.accepted
    assert abs(rec.tau - 50.0 * 0.1 ** rec.s) < 1e-12
    assert len(rec.trials) == rec.s + 1
    for tau, E in rec.trials[:-1]:
        assert E > C0 - p.rho1 * tau * rec.zz
    tau, E = rec.trials[-1]
    assert E <= C0 - p.rho1 * tau * rec.zz


def test_golden_small16_trajectory_unchanged():
    path = os.path.join(GOLD, "oracle_small16.json")
    gold = json.load(open(path))
    sys_, cfg = _small16()
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_)
    for rec_g in gold["steps"][:10]:
        rec = A.step()
        assert rec.s == rec_g["s"]
        assert abs(rec.E - rec_g["E"]) < 1e-11
        assert abs(rec.tau - rec_g["tau"]) < 1e-11 * rec_g["tau"]


# ---- modifications of section 3.3 (n_org, n_diag) and the residual of eq. "gra"

def _free_box(N, seed):
    n, L = 8, 5.0
    cfg = synth.custom("t", n, L, 0, 1.0, 0.5, N, seed_id=seed)
    sys_ = ks.System(n, L, np.zeros((0, 3)), np.zeros(0), np.zeros(0),
                     synth.occupations(cfg), ks.TERM_KIN)
    w = np.linalg.eigvalsh(dense.kinetic_matrix(n, L / n))
    return sys_, cfg, w


@pytest.mark.parametrize("n_org", [2, 3])
def test_orthonormalise_every_n_org_steps_reaches_dense_minimum(n_org):
    sys_, cfg, w = _free_box(7, 41)
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_, algm.Params(n_org=n_org))
    recs = A.run(4000, tol=1e-15)
    assert [r.orthonormalized for r in recs[:2 * n_org]] == [k % n_org == 0 for k in range(2 * n_org)]
    # finish on an orthonormalised iterate
    while A.l % n_org != 0:
        A.step()
    A.step()
    assert abs(A.E - 2 * np.sum(w[:7])) < 1e-10
    G = gram(A.W, A.h)
    assert np.max(np.abs(G - np.eye(7))) < 1e-12


def test_subspace_rotation_diagonalises_sigma_and_keeps_energy():
    sys_, cfg, w = _free_box(7, 43)
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_, algm.Params(n_diag=3))
    recs = [A.step() for _ in range(4)]
    assert [r.rotated for r in recs] == [True, False, False, True]
    E_before = A.terms.E
    S_before = A.sigma_full()
    S = A.sigma_full()
    off = S - np.diag(np.diag(S))
    assert np.max(np.abs(off)) < 1e-12 * np.max(np.abs(S))
    # E(W P) = E(W): the energy of the rotated iterate equals the accepted energy
    t, _, _ = ks.energy_and_h(A.W, sys_, A.vext)
    assert abs(t.E - A.E) < 1e-12 * abs(A.E)
    # the rotated block stays orthonormal and sigma holds the eigenvalues of Sigma
    assert np.max(np.abs(gram(A.W, A.h) - np.eye(7))) < 1e-12
    assert np.allclose(np.sort(A.sig), np.linalg.eigvalsh(0.5 * (S + S.T)), atol=1e-12)
    assert np.all(np.diff(A.sig) >= -1e-12)
    del E_before, S_before


def test_subspace_rotation_run_reaches_dense_minimum():
    sys_, cfg, w = _free_box(7, 47)
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_, algm.Params(n_diag=5, n_org=1))
    A.run(4000, tol=1e-15)
    assert abs(A.E - 2 * np.sum(w[:7])) < 1e-10


def test_subspace_rotation_needs_equal_occupations():
    sys_, cfg, _ = _free_box(2, 49)
    sys_.occ = np.array([2.0, 1.0])
    with pytest.raises(ValueError):
        algm.AlgorithmM(synth.orbitals(cfg), sys_, algm.Params(n_diag=4))


def test_residual_vanishes_on_exact_eigenvectors():
    """Plane waves are exact eigenvectors of the periodic FD Laplacian: for the
    free box the lowest 7 (constant, cos and sin along each axis) give
    H W = W Lambda, so the gradient of eq. "gra" is zero to rounding."""
    n, L = 8, 5.0
    h = L / n
    sys_ = ks.System(n, L, np.zeros((0, 3)), np.zeros(0), np.zeros(0), 2.0 * np.ones(7),
                     ks.TERM_KIN)
    x = h * np.arange(n)
    Zg, Yg, Xg = np.meshgrid(x, x, x, indexing="ij")
    k = 2 * np.pi / L
    fs = [np.ones_like(Xg)] + [f(k * c) for c in (Xg, Yg, Zg) for f in (np.cos, np.sin)]
    W = np.stack([f / np.sqrt(ks.inner(f, f, h)) for f in fs])
    A = algm.AlgorithmM(W, sys_, orthonormalize_start=False)
    assert A.residual() < 1e-12
    # and is not zero for a rotated-and-perturbed block
    rng = np.random.default_rng(3)
    B = algm.AlgorithmM(W + 0.1 * rng.standard_normal(W.shape), sys_)
    assert B.residual() > 1e-3


def test_residual_is_orthogonal_to_the_block_and_matches_the_trace_identity():
    sys_, cfg = _small16()
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_)
    A.step()
    N = A.W.shape[0]
    S = A.sigma_full()
    R = A.HW.reshape(N, -1) - S.T @ A.W.reshape(N, -1)
    # <W^T R> = 0 for orthonormal W (section 2.2: the gradient lies in the tangent space)
    WR = A.h ** 3 * A.W.reshape(N, -1) @ R.T
    assert np.max(np.abs(WR)) < 1e-10 * np.max(np.abs(S))
    # ||R||^2 = ||H W||^2 - ||Sigma||_F^2 for orthonormal W
    hw2 = A.h ** 3 * np.sum(A.HW * A.HW)
    assert abs(A.residual() ** 2 - (hw2 - np.sum(S * S))) < 1e-9 * hw2
