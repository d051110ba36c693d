"""Element-wise parity of the mixed form (FP32 orbitals and stencil, BF16 first
Gram, FP32-accurate second pass, FP64 Cholesky and reductions) with the FP64
oracle, at tolerances derived from the arithmetic (tests/_common.py):

  * the BF16 first-pass Gram and the FP32-accurate Gram (section 3.2) against
    the oracle's Gram of the same FP32 block;
  * the trial point W - tau Z (section 3.2) and its Gram, formed by the
    kernels a step uses;
  * single steps of Algorithm M from the same state: the oracle is handed the
    GPU's own previous iterates (as FP64), so trajectory drift does not enter;
    the backtracking exponent s is equal, tau_BB agrees to the bound the FP32
    directions allow, the new block agrees element by element, and the
    reported energy equals the oracle's energy of that block to the bound of
    the FP32 kinetic sums.

N = 512 runs on a 16^3 grid (4,096 points): the largest orbital count the
library admits, with every tile of the 512 x 512 Cholesky workspace and all
ten 128 x 128 block pairs of the Gram.
"""
import numpy as np
import pytest

import synth
from oracle import ks, orth as oorth, algm
from _common import (oracle_system, gpu_system, to_np, rel, gram_tolerance,
                     hamiltonian_error_bound, U32, UBF, LAM)
from _stepcheck import step_parity

pytestmark = pytest.mark.gpu

GRAM_CASES = [(16, 32), (100, 32), (128, 33), (144, 20), (300, 21), (512, 16)]


def _cfg(norb, n, seed):
    return synth.custom(f"mp_N{norb}_n{n}", n, 0.6 * n, max(1, min(norb // 2, 64)), 2.0, 0.5,
                        norb, min_sep=0.5, seed_id=seed)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _chunk(cfg):
    # FP32 runs of the Gram kernels: 64 points per chunk up to 128 orbitals,
    # whole split ranges above (bounded here by the grid)
    return 64 if cfg.norb <= 128 else cfg.ng


@pytest.mark.parametrize("norb,n", GRAM_CASES)
def test_gram_bf16_and_accurate_match_oracle(norb, n):
    cfg = _cfg(norb, n, 600 + norb)
    print(f"[gram] N={norb} n={n}", flush=True)
    so = oracle_system(cfg)
    W = _f32(oorth.orth(synth.orbitals(cfg), so.h)[0])
    g = gpu_system(cfg, "mixed")
    U = g.new_block(W)
    G_o = oorth.gram(W, so.h)
    G16 = g.gram(U, bf16=True)
    tol16 = gram_tolerance(W, so.h, _chunk(cfg), UBF)
    r16 = float(np.max(np.abs(G16 - G_o) / tol16))
    Gacc = g.gram(U)
    tola = gram_tolerance(W, so.h, _chunk(cfg), 0.0 if norb <= 128 else 2.0 ** -17)
    ra = float(np.max(np.abs(Gacc - G_o) / tola))
    print(f"[gram] N={norb}: bf16 max|dG| {np.max(np.abs(G16 - G_o)):.2e} ({r16:.3f} of bound), "
          f"accurate {np.max(np.abs(Gacc - G_o)):.2e} ({ra:.3f} of bound)", flush=True)
    assert r16 <= 1.0
    assert ra <= 1.0
    # the BF16 bound is tight enough to see a lost 64-point chunk of one orbital pair
    A = W.reshape(norb, -1)
    lost = so.h ** 3 * np.abs(A[:, :64] @ A[:, :64].T)
    assert np.any(lost > tol16)


@pytest.mark.parametrize("prec,norb,n", [("mixed", 16, 32), ("mixed", 128, 33),
                                         ("mixed", 144, 20), ("mixed", 512, 16),
                                         ("fp64", 40, 24), ("fp64", 200, 19)])
def test_trial_point_matches_oracle(prec, norb, n):
    cfg = _cfg(norb, n, 700 + norb)
    print(f"[trial] {prec} N={norb} n={n}", flush=True)
    so = oracle_system(cfg)
    W = oorth.orth(synth.orbitals(cfg), so.h)[0]
    if prec == "mixed":
        W = _f32(W)
    g = gpu_system(cfg, prec)
    U = g.new_block(W)
    tau = 0.5 / algm.lambda_max_kinetic(so.h)
    Wt, G = g.trial_point(U, tau)
    Wt = to_np(Wt).astype(np.float64)
    terms, HW, sig = ks.energy_and_h(W, so)
    Wt_o = W - tau * (HW - sig[:, None, None, None] * W)
    if prec == "fp64":
        assert rel(Wt, Wt_o) < 1e-12
        assert rel(G, oorth.gram(Wt, so.h)) < 1e-13
        return
    veff = ks.potentials(W, so)[3]
    dH = hamiltonian_error_bound(W, veff, so.h)
    # tau (H u) error, the FP32 sigma_ii (its sums: LAM sqrt(n) U32 relative at most)
    # and three roundings of the FP32 result
    dsig = LAM * np.sqrt(cfg.ng) * U32 * np.abs(sig)
    tolW = (tau * dH + tau * dsig[:, None, None, None] * np.abs(W)
            + 3 * U32 * (np.abs(W) + tau * np.abs(HW)))
    rW = float(np.max(np.abs(Wt - Wt_o) / tolW))
    bf16 = True  # two passes: the first Gram is the BF16 one
    tolG = gram_tolerance(Wt, so.h, _chunk(cfg), UBF if bf16 else 0.0)
    rG = float(np.max(np.abs(G - oorth.gram(Wt, so.h)) / tolG))
    print(f"[trial] N={norb}: W~ {np.max(np.abs(Wt - Wt_o)):.2e} ({rW:.3f} of bound), "
          f"G {np.max(np.abs(G - oorth.gram(Wt, so.h))):.2e} ({rG:.3f} of bound)", flush=True)
    assert rW <= 1.0
    assert rG <= 1.0


# N = 20, 64, 72, 90 take the remaining row-tile counts (2, 4, 5, 6) of the
# N <= 128 fused apply + Gram and FP32 apply kernels
@pytest.mark.parametrize("norb,n", [(16, 32), (48, 27), (128, 33), (144, 20), (512, 16),
                                    (20, 24), (64, 22), (72, 21), (90, 24)])
def test_mixed_steps_from_same_state(norb, n):
    cfg = _cfg(norb, n, 800 + norb)
    print(f"[mixed step] N={norb} n={n}", flush=True)
    step_parity(cfg, 3, f"mixed N={norb} n={n}")


def test_fp64_512_orbitals_follow_oracle():
    """N = 512 in FP64 on 16^3 points: Gram, Householder-QR factor and three
    steps of Algorithm M against the oracle at FP64 tolerances."""
    cfg = _cfg(512, 16, 900)
    print("[fp64 N=512]", flush=True)
    so = oracle_system(cfg)
    X = synth.orbitals(cfg)
    p = algm.Params()
    p.tau_init = 1.0 / algm.lambda_max_kinetic(so.h)
    g = gpu_system(cfg, "fp64", tau_init=p.tau_init)
    U = g.new_block(X)
    assert rel(g.gram(U), oorth.gram(X, so.h)) < 1e-13
    err = g.orthonormalize_(U)
    W_o, _ = oorth.orth(X, so.h)
    assert err < 1e-12
    assert rel(to_np(U), W_o) < 1e-9
    A = algm.AlgorithmM(W_o, so, p, orthonormalize_start=False)
    U = g.new_block(W_o)
    for k in range(3):
        r = A.step()
        info = g.step_(U)
        print(f"[fp64 N=512] step {k}: s {info['s']}/{r.s} E {info['E']:.12f}/{r.E:.12f}",
              flush=True)
        assert info["s"] == r.s
        assert abs(info["E"] - r.E) < 1e-9 * max(1, abs(r.E))
        assert abs(info["tau_bb"] - r.tau_bb) < 1e-7 * r.tau_bb
    assert rel(to_np(U), A.W) < 1e-8


def test_mixed_512_orthonormalize_matches_householder():
    cfg = _cfg(512, 16, 901)
    so = oracle_system(cfg)
    X = _f32(synth.orbitals(cfg))
    g = gpu_system(cfg, "mixed")
    U = g.new_block(X)
    err = g.orthonormalize_(U)
    W_o, _ = oorth.orth(X, so.h)
    d = float(np.max(np.abs(to_np(U) - W_o)))
    print(f"[mixed N=512] orth err {err:.2e}, |U - Q| {d:.2e}", flush=True)
    assert err < 1e-5
    assert rel(to_np(U), W_o) < 1e-4


def test_mixed_one_pass_is_fp32_accurate_above_128():
    """orth_passes = 1 in mixed precision above 128 orbitals: the only pass
    must use the FP32-accurate Gram, so the steps stay orthonormal to the FP32
    level (a BF16 Gram in the single pass leaves ~1e-3)."""
    cfg = _cfg(144, 20, 902)
    so = oracle_system(cfg)
    W0 = _f32(oorth.orth(synth.orbitals(cfg), so.h)[0])
    g = gpu_system(cfg, "mixed", orth_passes=1)
    U = g.new_block(W0)
    for k in range(4):
        info = g.step_(U)
        assert np.isfinite(info["E"])
    dev = float(np.max(np.abs(oorth.gram(to_np(U).astype(np.float64), so.h) - np.eye(144))))
    print(f"[one pass N=144] orthonormality {dev:.2e}", flush=True)
    assert dev < 1e-5
