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
