"""Mixed precision (FP32 orbitals and stencil, BF16 first Gram, FP32 second
Gram and apply, FP64 Cholesky and reductions) against FP64 and the oracle.

Targets stated for the method: energies within 1e-6 Ha of the FP64 result
after FP64 refinement, orthonormality error <= 1e-10 after refinement.
"""
import numpy as np
import pytest

import synth
from oracle import ks, orth as oorth, algm
from _common import oracle_system, gpu_system, to_np, rel

pytestmark = pytest.mark.gpu


def _run(g, U, tol, max_steps):
    df = []
    info = None
    for k in range(max_steps):
        info = g.step_(U)
        df.append(info["df"])
        if len(df) >= 3 and np.mean(df[-3:]) < tol:
            return info, k + 1, True
    return info, max_steps, False


def test_mixed_energy_and_orth_match_fp64():
    cfg = synth.CONFIGS["fp64_48"]
    so = oracle_system(cfg)
    W = oorth.orth(synth.orbitals(cfg), so.h)[0]
    e_o = ks.energy(W, so).E
    g32 = gpu_system(cfg, "mixed")
    U32 = g32.new_block(W)
    e32 = g32.energy(U32)["E"]
    print(f"[mixed] E oracle {e_o:.12f} mixed {e32:.12f} rel {abs(e32 - e_o) / abs(e_o):.2e}")
    assert abs(e32 - e_o) < 2e-6 * abs(e_o)
    X = synth.orbitals(cfg)
    Ux = g32.new_block(X)
    err = g32.orthonormalize_(Ux)
    assert err < 1e-6
    assert rel(to_np(Ux), oorth.orth(X, so.h)[0]) < 1e-4


def test_mixed_then_refined_reaches_fp64_minimum():
    """fp64_48: mixed steps, FP64 refinement; |E - E_fp64| <= 1e-6 Ha."""
    import paper_1510_07230_amd as pk
    cfg = synth.CONFIGS["fp64_48"]
    so = oracle_system(cfg)
    W = oorth.orth(synth.orbitals(cfg), so.h)[0]
    g64 = gpu_system(cfg, "fp64")
    U64 = g64.new_block(W)
    i64, k64, c64 = _run(g64, U64, 1e-13, 6000)
    g32 = gpu_system(cfg, "mixed")
    U32 = g32.new_block(W)
    i32, k32, _ = _run(g32, U32, 1e-9, 3000)
    gr = gpu_system(cfg, "fp64")
    Ur = gr.new_block()
    gr.convert(U32, Ur)
    gr.orthonormalize_(Ur)
    ir, kr, cr = _run(gr, Ur, 1e-13, 6000)
    G = gr.gram(Ur)
    orth_err = float(np.max(np.abs(G - np.eye(cfg.norb))))
    print(f"[mixed] fp64 {i64['E']:.12f} ({k64} steps, conv {c64}); mixed {i32['E']:.12f} "
          f"({k32}); refined {ir['E']:.12f} ({kr}, conv {cr}); orth {orth_err:.2e}")
    assert c64 and cr
    assert abs(ir["E"] - i64["E"]) <= 1e-6
    assert orth_err <= 1e-10


def test_converged_energy_matches_oracle_small16():
    cfg = synth.CONFIGS["small16"]
    so = oracle_system(cfg)
    A = algm.AlgorithmM(synth.orbitals(cfg), so)
    A.run(3000, tol=1e-13)
    g = gpu_system(cfg, "fp64")
    U = g.new_block(synth.orbitals(cfg))
    g.orthonormalize_(U)
    info, k, conv = _run(g, U, 1e-13, 3000)
    g32 = gpu_system(cfg, "mixed")
    U32 = g32.new_block(synth.orbitals(cfg))
    g32.orthonormalize_(U32)
    i32, _, _ = _run(g32, U32, 1e-9, 3000)
    gr = gpu_system(cfg, "fp64")
    Ur = gr.new_block()
    gr.convert(U32, Ur)
    gr.orthonormalize_(Ur)
    ir, _, cr = _run(gr, Ur, 1e-13, 3000)
    print(f"[conv] oracle {A.E:.12f} gpu {info['E']:.12f} refined {ir['E']:.12f}")
    assert conv and cr
    assert abs(info["E"] - A.E) <= 1e-6
    assert abs(ir["E"] - A.E) <= 1e-6


@pytest.mark.parametrize("norb", [16, 40, 100, 128])
def test_mixed_steps_follow_oracle_every_tile_count(norb):
    """Mixed steps for orbital counts that leave 0..3 row tiles and part of the
    last 32-orbital chunk empty in the fused apply + second Gram: the energies
    follow the oracle's trajectory to the FP32 level and the block stays
    orthonormal (no padding value leaks into the result)."""
    cfg = synth.custom(f"mixed_N{norb}", 32, 14.0, max(1, norb // 2), 2.0, 0.5, norb,
                       min_sep=1.0, seed_id=300 + norb)
    so = oracle_system(cfg)
    W = oorth.orth(synth.orbitals(cfg), so.h)[0]
    A = algm.AlgorithmM(W, so)
    g32 = gpu_system(cfg, "mixed")
    U32 = g32.new_block(W)
    for k in range(4):
        ref = A.step()
        info = g32.step_(U32)
        assert np.isfinite(info["E"])
        print(f"[mixed N={norb}] step {k}: oracle {ref.E:.10f} mixed {info['E']:.10f}")
        assert abs(info["E"] - ref.E) < 2e-6 * abs(ref.E)
    G = g32.gram(U32)
    assert np.all(np.isfinite(G))
    assert np.max(np.abs(G - np.eye(norb))) < 1e-5


@pytest.mark.parametrize("norb,n", [(48, 27), (40, 25)])
def test_mixed_steps_follow_oracle_ragged_grid(norb, n):
    """Mixed steps on grids whose point count is not a multiple of the 32- and
    64-point blocks and whose side is not a multiple of the 32-point stencil
    tile: the last block of the apply, the trial + Gram and the fused apply +
    Gram takes the element-tested path, the stencil stores its points beyond
    the grid outside the plane range, and N = 48 has every row of its tiles
    inside the problem while N = 40 does not.  The energies follow the
    oracle's trajectory to the FP32 level and the block stays orthonormal."""
    cfg = synth.custom(f"mixed_ragged_N{norb}_n{n}", n, 0.44 * n, max(1, norb // 2), 2.0, 0.5,
                       norb, min_sep=1.0, seed_id=500 + norb)
    print(f"[mixed ragged] N={norb} n={n} ng={n ** 3}", flush=True)
    so = oracle_system(cfg)
    W = oorth.orth(synth.orbitals(cfg), so.h)[0]
    A = algm.AlgorithmM(W, so)
    g32 = gpu_system(cfg, "mixed")
    U32 = g32.new_block(W)
    for k in range(4):
        ref = A.step()
        info = g32.step_(U32)
        assert np.isfinite(info["E"])
        print(f"[mixed ragged N={norb} n={n}] step {k}: oracle {ref.E:.10f} mixed {info['E']:.10f}")
        assert abs(info["E"] - ref.E) < 2e-6 * abs(ref.E)
    G = g32.gram(U32)
    assert np.all(np.isfinite(G))
    assert np.max(np.abs(G - np.eye(norb))) < 1e-5


@pytest.mark.parametrize("norb,n", [(144, 20), (200, 19), (257, 24), (300, 21)])
def test_mixed_more_than_128_orbitals_follow_oracle(norb, n):
    """N > 128 in mixed precision (128 x 128 block Gram on BF16 / split-BF16
    MFMA, split-BF16 triangular apply): row blocks that end inside a 32-orbital
    chunk or a 16-orbital tile, and grids whose point count is not a multiple of
    4 (scalar loads) or of 32 (ragged last chunk).  The Gram matches the oracle
    to the split-BF16 level, orthonormalisation reproduces the oracle's QR
    factor and four steps follow the oracle's energies to the FP32 level."""
    cfg = synth.custom(f"mixed_big_N{norb}", n, 0.6 * n, max(1, norb // 2), 2.0, 0.5, norb,
                       min_sep=0.5, seed_id=400 + norb)
    print(f"[mixed big] N={norb} n={n}", flush=True)
    so = oracle_system(cfg)
    X = synth.orbitals(cfg)
    g32 = gpu_system(cfg, "mixed")
    Ux = g32.new_block(X)
    G = g32.gram(Ux)
    G_o = oorth.gram(X, so.h)
    assert rel(G, G_o) < 2e-6
    err = g32.orthonormalize_(Ux)
    W_o, _ = oorth.orth(X, so.h)
    assert err < 1e-5
    assert rel(to_np(Ux), W_o) < 1e-4
    A = algm.AlgorithmM(W_o, so, orthonormalize_start=False)
    U32 = g32.new_block(W_o)
    for k in range(4):
        ref = A.step()
        info = g32.step_(U32)
        print(f"[mixed big N={norb}] step {k}: oracle {ref.E:.10f} mixed {info['E']:.10f} "
              f"s {ref.s}/{info['s']}", flush=True)
        assert np.isfinite(info["E"])
        assert abs(info["E"] - ref.E) < 2e-6 * abs(ref.E)
    G = g32.gram(U32)
    assert np.all(np.isfinite(G))
    assert np.max(np.abs(G - np.eye(norb))) < 1e-5
