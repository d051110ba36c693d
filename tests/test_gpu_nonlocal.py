"""The nonlocal part of the pseudopotential (section 2.1, V_nloc u = sum_l
<xi_l, u> xi_l, four Gaussian projectors per ion) on the GPU against the
oracle: energy terms, H U and sigma, trajectories, the gradient and the forces
in FP64, and mixed steps from the same state.  Grids where each ion's cube is
smaller than the grid (n = 32, 27) and where it covers the whole grid (n = 12)."""
import numpy as np
import pytest

import synth
from oracle import ks, orth as oorth, algm
from _common import oracle_system, gpu_system, to_np, rel
from _stepcheck import step_parity

pytestmark = pytest.mark.gpu

CASES = [
    synth.custom("nl32", 32, 14.0, 5, 2.0, 0.5, 6, min_sep=1.5, seed_id=71),
    synth.custom("nl27", 27, 11.0, 4, (1.0, 2.0), (0.45, 0.6), 5, min_sep=1.5, seed_id=72),
    synth.custom("nl12", 12, 6.0, 2, 2.0, 0.5, 3, seed_id=73),
]


def _setup(cfg, prec="fp64", **params):
    pp = synth.projector_params(cfg)
    so = oracle_system(cfg, proj=pp)
    W = oorth.orth(synth.orbitals(cfg), so.h)[0]
    g = gpu_system(cfg, prec, proj=pp, **params)
    return pp, so, W, g


@pytest.mark.parametrize("cfg", CASES, ids=lambda c: c.name)
def test_nonlocal_energy_and_hamiltonian(cfg):
    print(f"[nloc] {cfg.name}", flush=True)
    pp, so, W, g = _setup(cfg)
    U = g.new_block(W)
    e = g.energy(U)
    t = ks.energy(W, so)
    assert t.E_nl > 1e-3
    assert abs(e["E_nl"] - t.E_nl) < 1e-11 * max(1.0, t.E_nl)
    assert abs(e["E"] - t.E) < 1e-9 * max(1.0, abs(t.E))
    HU, sig = g.hamiltonian(U)
    veff = ks.potentials(W, so)[3]
    HU_o = ks.hamiltonian_apply_fixed(W, veff, so.h, Xi=ks.projectors(so))
    assert rel(to_np(HU), HU_o) < 1e-11
    assert np.max(np.abs(sig - ks.inner(W, HU_o, so.h))) < 1e-10
    # removing the projectors restores the local model
    g.set_projectors(None)
    e0 = g.energy(U)
    assert e0["E_nl"] == 0.0
    assert abs(e0["E"] - (t.E - t.E_nl)) < 1e-9 * max(1.0, abs(t.E))


def test_nonlocal_trajectory_fp64():
    cfg = CASES[0]
    pp, so, W, g0 = _setup(cfg)
    p = algm.Params()
    p.tau_init = 1.0 / algm.lambda_max_kinetic(so.h)
    g = gpu_system(cfg, "fp64", proj=pp, tau_init=p.tau_init)
    A = algm.AlgorithmM(W, so, p, orthonormalize_start=False)
    U = g.new_block(W)
    for k in range(6):
        r = A.step()
        info = g.step_(U)
        print(f"[nloc traj] step {k}: s {info['s']}/{r.s} E {info['E']:.12f}/{r.E:.12f}",
              flush=True)
        assert info["s"] == r.s
        assert abs(info["E"] - r.E) < 1e-9 * max(1.0, abs(r.E))
        assert abs(info["tau_bb"] - r.tau_bb) < 1e-7 * r.tau_bb
    assert rel(to_np(U), A.W) < 1e-8


@pytest.mark.parametrize("cfg", CASES[:2] + [CASES[2]], ids=lambda c: c.name)
def test_nonlocal_gradient_and_forces(cfg):
    pp, so, W, g = _setup(cfg)
    U = g.new_block(W)
    g.energy(U)
    dU, dR, ds = g.backward(U, gE=1.0)
    assert rel(to_np(dU), ks.energy_gradient(W, so)) < 1e-10
    dR_o, ds_o = ks.forces(W, so)
    assert rel(to_np(dR), dR_o) < 1e-9
    assert rel(to_np(ds), ds_o) < 1e-9
    # the nonlocal share of the force is not negligible here
    so_loc = oracle_system(cfg)
    dR_loc, _ = ks.forces(W, so_loc)
    assert np.max(np.abs(dR_o - dR_loc)) > 1e-3 * np.max(np.abs(dR_o))


def test_nonlocal_more_than_128_orbitals_fp64():
    cfg = synth.custom("nl144", 20, 9.0, 6, 2.0, 0.5, 144, min_sep=1.5, seed_id=74)
    pp, so, W, g = _setup(cfg)
    U = g.new_block(W)
    e = g.energy(U)
    t = ks.energy(W, so)
    assert abs(e["E"] - t.E) < 1e-9 * max(1.0, abs(t.E))
    assert abs(e["E_nl"] - t.E_nl) < 1e-11 * max(1.0, t.E_nl)


@pytest.mark.parametrize("norb,n", [(16, 32), (144, 20)])
def test_nonlocal_mixed_steps_from_same_state(norb, n):
    cfg = synth.custom(f"nlm_N{norb}", n, 0.6 * n, max(1, min(norb // 2, 24)), 2.0, 0.5, norb,
                       min_sep=1.0, seed_id=880 + norb)
    step_parity(cfg, 3, f"nloc mixed N={norb}", proj=synth.projector_params(cfg))
