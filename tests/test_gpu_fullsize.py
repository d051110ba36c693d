"""Parity at the benchmark's full size (96^3 grid, N = 128, 64 ions) in the
launch configuration bench.py times: sampled outputs the oracle can compute,
and one Algorithm-M step against the oracle."""
import numpy as np
import pytest

import synth
from oracle import ks, orth as oorth, algm
from _common import oracle_system, gpu_system, to_np, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    cfg = synth.CONFIGS["mixed96"]
    so = oracle_system(cfg)
    W = oorth.orth(synth.orbitals(cfg), so.h)[0]
    return cfg, so, W


def test_fullsize_energy_fields_and_sampled_hamiltonian(setup):
    cfg, so, W = setup
    print("[full] energy + fields + sampled H u", flush=True)
    rho, VH, vx, veff, ex, vext, _ = ks.potentials(W, so)
    terms = ks.energy(W, so, vext)
    g = gpu_system(cfg, "fp64")
    U = g.new_block(W)
    e = g.energy(U)
    assert abs(e["E"] - terms.E) < 1e-9 * abs(terms.E)
    f = g.fields()
    assert rel(to_np(f["veff"]), veff) < 1e-11
    HU, sig = g.hamiltonian(U)
    for i in (0, 37, 127):
        hu_o = ks.hamiltonian_apply_fixed(W[i:i + 1], veff, so.h)[0]
        assert rel(to_np(HU[i]), hu_o) < 1e-11
    g32 = gpu_system(cfg, "mixed")
    U32 = g32.new_block(W)
    e32 = g32.energy(U32)
    assert abs(e32["E"] - terms.E) < 2e-6 * abs(terms.E)
    HU32, _ = g32.hamiltonian(U32)
    hu_o = ks.hamiltonian_apply_fixed(W[5:6], veff, so.h)[0]
    assert rel(to_np(HU32[5]), hu_o) < 1e-4


def test_fullsize_first_step_matches_oracle(setup):
    cfg, so, W = setup
    print("[full] first step", flush=True)
    p = algm.Params()
    p.tau_init = 1.0 / algm.lambda_max_kinetic(so.h)
    A = algm.AlgorithmM(W, so, p, orthonormalize_start=False)
    r = A.step()
    g = gpu_system(cfg, "fp64", tau_init=p.tau_init)
    U = g.new_block(W)
    info = g.step_(U)
    assert info["s"] == r.s
    assert abs(info["E"] - r.E) < 1e-9 * abs(r.E)
    assert abs(info["zz"] - r.zz) < 1e-8 * r.zz
    Wn = to_np(U)
    for i in (0, 64, 127):
        assert rel(Wn[i], A.W[i]) < 1e-9


def test_fullsize_mixed_steps_match_oracle():
    """Two mixed steps at 96^3 x 128 (the benchmark's configuration and launch
    shapes) against the oracle from the same state: s equal, tau_BB within the
    FP32-direction bound, the new block element-wise and the reported energy
    against the oracle's energy of that block (bounds in tests/_common.py)."""
    from _stepcheck import step_parity
    cfg = synth.CONFIGS["mixed96"]
    print("[full] mixed steps", flush=True)
    step_parity(cfg, 2, "full mixed96")
