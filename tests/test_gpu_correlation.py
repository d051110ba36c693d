"""LDA correlation (opt-in term POU_TERM_CORR, Perdew-Zunger form) on the GPU
against the oracle: fields, energy terms, H U, the energy gradient and a
short trajectory."""
import numpy as np
import pytest

import synth
from oracle import ks, algm, orth as oorth
from _common import gpu_system, to_np, rel

pytestmark = pytest.mark.gpu

TERMS = ks.TERM_ALL | ks.TERM_CORR

CASES = [
    synth.CONFIGS["small16"],
    synth.custom("ragged27c", 27, 9.0, 3, (1.0, 2.0), (0.45, 0.7), 5, min_sep=1.5, seed_id=141),
]


def _oracle(cfg):
    R, Z, s = synth.atoms(cfg)
    return ks.System(cfg.n, cfg.L, R, Z, s, synth.occupations(cfg), TERMS)


@pytest.mark.parametrize("cfg", CASES, ids=lambda c: c.name)
def test_correlation_fields_energy_hamiltonian(cfg):
    print(f"[corr] {cfg.name}", flush=True)
    so = _oracle(cfg)
    W = oorth.orth(synth.orbitals(cfg), so.h)[0]
    g = gpu_system(cfg, terms=TERMS)
    U = g.new_block(W)
    e = g.energy(U)
    rho, VH, vxc, veff, ex, vext, ec = ks.potentials(W, so)
    t = ks.energy(W, so, vext)
    assert t.E_c < 0.0
    for k in ("E", "E_kin", "E_ext", "E_H", "E_x", "E_c"):
        assert abs(e[k] - getattr(t, k)) < 1e-9 * max(1.0, abs(t.E)), (k, e[k], getattr(t, k))
    assert rel(to_np(g.fields()["veff"]), veff) < 1e-11
    HU, sig = g.hamiltonian(U)
    HU_o = ks.hamiltonian_apply_fixed(W, veff, so.h)
    assert rel(to_np(HU), HU_o) < 1e-11


def test_correlation_gradient_matches_oracle_and_differences():
    cfg = CASES[1]
    so = _oracle(cfg)
    U0 = synth.orbitals(cfg) * 0.05
    g = gpu_system(cfg, terms=TERMS)
    U = g.new_block(U0)
    dU, _, _ = g.backward(U)
    G_o = ks.energy_gradient(U0, so)
    assert rel(to_np(dU), G_o) < 1e-10


def test_correlation_trajectory_follows_oracle():
    print("[corr] trajectory", flush=True)
    cfg = CASES[0]
    so = _oracle(cfg)
    p = algm.Params()
    p.tau_init = 1.0 / algm.lambda_max_kinetic(so.h)
    A = algm.AlgorithmM(synth.orbitals(cfg), so, p)
    g = gpu_system(cfg, terms=TERMS, tau_init=p.tau_init)
    U = g.new_block(A.W)
    for k in range(10):
        r = A.step()
        info = g.step_(U)
        assert info["s"] == r.s, k
        assert abs(info["E"] - r.E) < 1e-9 * max(1.0, abs(r.E)), (k, info["E"], r.E)
