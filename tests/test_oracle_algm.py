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


# ---- Barzilai-Borwein values, their alternation, and the C/Q recursion
# (section 3.2), pinned by hand-known traces and closed forms

def _plane_wave_pair(n=8, L=5.0):
    """Two functions orthonormal in the grid inner product h^3 sum a b:
    normalised cos and sin of the lowest x mode (exactly orthogonal on the grid)."""
    h = L / n
    x = h * np.arange(n)
    c = np.broadcast_to(np.cos(2 * np.pi * x / L)[None, None, :], (n, n, n)).copy()
    s = np.broadcast_to(np.sin(2 * np.pi * x / L)[None, None, :], (n, n, n)).copy()
    e1 = c / np.sqrt(h ** 3 * np.sum(c * c))
    e2 = s / np.sqrt(h ** 3 * np.sum(s * s))
    return e1, e2, h


def _free_runner(n=8, L=5.0, N=2, **params):
    cfg = synth.custom("t", n, L, 0, 1.0, 0.5, N, seed_id=61)
    sys_ = ks.System(n, L, np.zeros((0, 3)), np.zeros(0), np.zeros(0),
                     synth.occupations(cfg), ks.TERM_KIN)
    return algm.AlgorithmM(synth.orbitals(cfg), sys_, algm.Params(**params))


# S = [a1 e1, a2 e2], Y = [b1 e1 + c1 e2, b2 e2]:
#   tr<S^T S> = a1^2 + a2^2, tr<S^T Y> = a1 b1 + a2 b2, tr<Y^T Y> = b1^2 + c1^2 + b2^2
BB_CASES = [
    # (a1, a2, b1, c1, b2)
    (2.0, 1.0, 0.5, 1.0, 0.25),
    (0.3, -1.5, -2.0, 0.7, 0.4),     # tr<S^T Y> < 0: its absolute value is used
    (1e-3, 2e-3, 5e-2, -3e-2, 1e-2),
]


def _bb_blocks(a1, a2, b1, c1, b2):
    e1, e2, h = _plane_wave_pair()
    S = np.stack([a1 * e1, a2 * e2])
    Y = np.stack([b1 * e1 + c1 * e2, b2 * e2])
    ss = a1 * a1 + a2 * a2
    sy = a1 * b1 + a2 * b2
    yy = b1 * b1 + c1 * c1 + b2 * b2
    return S, Y, ss, sy, yy


@pytest.mark.parametrize("case", BB_CASES)
def test_bb_values_from_hand_known_traces(case):
    """tau1 = tr<S^T S>/|tr<S^T Y>| and tau2 = |tr<S^T Y>|/tr<Y^T Y> (section 3.2)
    on blocks whose traces are known by construction; fixed modes 1 and 2, and
    the alternating mode 0 (tau1 on odd l, tau2 on even l)."""
    S, Y, ss, sy, yy = _bb_blocks(*case)
    tau1 = ss / abs(sy)
    tau2 = abs(sy) / yy
    assert abs(tau1 - tau2) > 1e-3 * tau1      # the cases tell the two values apart
    A1 = _free_runner(bb_mode=1)
    A2 = _free_runner(bb_mode=2)
    A0 = _free_runner(bb_mode=0)
    for l in (1, 2, 3, 4, 7):
        assert abs(A1._bb_value(S, Y, l) - tau1) < 1e-13 * tau1
        assert abs(A2._bb_value(S, Y, l) - tau2) < 1e-13 * tau2
        want = tau1 if l % 2 == 1 else tau2
        assert abs(A0._bb_value(S, Y, l) - want) < 1e-13 * want, l


def test_bb_step_uses_the_last_two_iterates_and_directions():
    """bb_step forms S = W^(l) - W^(l-1) and Y = Z^(l) - Z^(l-1) from the stored
    history: plant a history whose differences are the hand-known blocks."""
    S, Y, ss, sy, yy = _bb_blocks(*BB_CASES[0])
    A = _free_runner(bb_mode=0)
    rng = np.random.default_rng(7)
    Z = rng.standard_normal(A.W.shape)
    A.Wp = A.W - S
    A.Zp = Z - Y
    A.l = 1
    assert abs(A.bb_step(Z) - ss / abs(sy)) < 1e-12 * ss / abs(sy)
    A.l = 2
    assert abs(A.bb_step(Z) - abs(sy) / yy) < 1e-12 * abs(sy) / yy
    # l = 0 (no history) takes tau_init whatever is stored
    A.l = 0
    assert A.bb_step(Z) == A.tau_init


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_bb_fallback_on_zero_or_nonfinite_values(mode):
    """No usable BB value (S = 0 or Y = 0 make a ratio 0/0, x/0 or 0) falls back
    to tau_init (the reading for a missing safeguard)."""
    S, Y, _, _, _ = _bb_blocks(*BB_CASES[0])
    A = _free_runner(bb_mode=mode, tau_init=0.0123)
    zero = np.zeros_like(S)
    for l in (1, 2):
        assert A._bb_value(zero, Y, l) == 0.0123
        assert A._bb_value(S, zero, l) == 0.0123
        assert A._bb_value(zero, zero, l) == 0.0123
    # S and Y in different orbitals: tr<S^T Y> = 0 exactly, so tau1 = x/0 and tau2 = 0
    e1, e2, _ = _plane_wave_pair()
    So = np.stack([e1, np.zeros_like(e1)])
    Yo = np.stack([np.zeros_like(e2), e2])
    for l in (1, 2):
        assert A._bb_value(So, Yo, l) == 0.0123


def test_bb_alternation_along_a_trajectory():
    """Along a run with mode 0, each step's tau_BB is the value the paper's
    formula gives for the recorded W^(l), W^(l-1), Z^(l), Z^(l-1): tau1 on odd l,
    tau2 on even l, tau_init at l = 0 (traces summed here with plain numpy)."""
    sys_, cfg = _small16()
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_, algm.Params(bb_mode=0))
    h3 = sys_.h ** 3
    Ws, Zs = [], []
    for l in range(16):
        Ws.append(A.W.copy())
        Zs.append(A.direction())
        rec = A.step()
        if l == 0:
            assert rec.tau_bb == A.tau_init
            continue
        S = Ws[l] - Ws[l - 1]
        Y = Zs[l] - Zs[l - 1]
        ss = h3 * float(np.sum(S * S))
        sy = abs(h3 * float(np.sum(S * Y)))
        yy = h3 * float(np.sum(Y * Y))
        want = ss / sy if l % 2 == 1 else sy / yy
        assert abs(rec.tau_bb - want) < 1e-9 * want, (l, rec.tau_bb, want)


@pytest.mark.parametrize("eta", [0.0, 0.85, 1.0])
def test_nonmonotone_reference_matches_closed_form(eta):
    """Q^(0) = 1, Q^(l+1) = eta Q^(l) + 1 and C^(l+1) = (eta Q^(l) C^(l) + E^(l+1)) / Q^(l+1)
    (section 3.2) unroll to Q^(l) = sum_{j<=l} eta^j and
    C^(l) = sum_{j<=l} eta^(l-j) E^(j) / Q^(l): a weighted mean of the energies.
    eta = 0 gives C = E, eta = 1 the running mean."""
    sys_, cfg = _small16()
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_, algm.Params(eta=eta))
    E = [A.E]
    for l in range(1, 51):
        rec = A.step()
        E.append(rec.E)
        w = np.array([eta ** (l - j) for j in range(l + 1)])
        Q = float(np.sum(w))
        C = float(np.sum(w * np.array(E))) / Q
        assert abs(rec.Q - Q) < 1e-12 * Q, (l, rec.Q, Q)
        assert abs(rec.C - C) < 1e-12 * abs(C), (l, rec.C, C)
        if eta == 0.0:
            assert rec.C == rec.E
        if eta == 1.0:
            assert abs(rec.C - np.mean(E)) < 1e-12 * abs(rec.C)


def test_linear_problem_with_nonlocal_projectors_reaches_dense_minimum():
    """K + V_ext + V_nloc on a 10^3 grid: Algorithm M reaches the sum of the
    lowest eigenvalues of the dense matrix (V_nloc built as h^3 Xi^T Xi)."""
    cfg = synth.custom("tnl", 10, 6.0, 2, (1.0, 2.0), (0.45, 0.7), 2, seed_id=9)
    R, Z, s = synth.atoms(cfg)
    sys_ = ks.System(10, 6.0, R, Z, s, synth.occupations(cfg),
                     ks.TERM_KIN | ks.TERM_EXT | ks.TERM_NLOC, proj=synth.projector_params(cfg))
    Emin, w = dense.linear_minimum(sys_)
    E0, _ = dense.linear_minimum(ks.System(10, 6.0, R, Z, s, synth.occupations(cfg),
                                           ks.TERM_KIN | ks.TERM_EXT))
    assert Emin > E0 + 1e-3  # the projectors are repulsive and felt
    assert w[2] - w[1] > 1e-2
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_)
    A.run(4000, tol=1e-15)
    assert abs(A.E - Emin) < 1e-10
