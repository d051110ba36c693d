"""The non-allocating Gram entry point (pou_gram_static) against the
context's pou_gram, through the C ABI: two calls in a row on one device, the
second with a smaller block, in FP64 and in mixed precision (FP32-accurate and
BF16 first-pass Gram).  Both must match the oracle's Gram of the same block to
the bounds derived for their arithmetic, and each other to the sum of those
bounds (the two paths split the grid into different numbers of ranges)."""
import numpy as np
import pytest

import synth
from oracle import orth as oorth
from _common import oracle_system, gpu_system, to_np, rel, gram_tolerance, UBF

pytestmark = pytest.mark.gpu


def _case(norb, n, seed):
    return synth.custom(f"na_N{norb}_n{n}", n, 0.6 * n, 2, 2.0, 0.5, norb, seed_id=seed)


@pytest.mark.parametrize("prec", ["fp64", "mixed", "mixed-bf16"])
def test_gram_static_matches_context_gram(prec):
    import torch
    import paper_1510_07230_amd as pk
    bf16 = prec == "mixed-bf16"
    for norb, n in ((128, 40), (37, 21)):  # the second call is smaller in both N and ng
        cfg = _case(norb, n, 950 + norb)
        print(f"[no-alloc] {prec} N={norb} n={n}", flush=True)
        so = oracle_system(cfg)
        X = oorth.orth(synth.orbitals(cfg), so.h)[0]
        g = gpu_system(cfg, "fp64" if prec == "fp64" else "mixed")
        U = g.new_block(X)
        Xb = to_np(U).astype(np.float64)
        G_ctx = g.gram(U, bf16=bf16)
        G_st = to_np(pk.gram_static(U, so.h ** 3, bf16=bf16))
        torch.cuda.synchronize()
        G_o = oorth.gram(Xb, so.h)
        if prec == "fp64":
            assert rel(G_st, G_o) < 1e-13
            assert rel(G_st, G_ctx) < 1e-13
        else:
            tol = gram_tolerance(Xb, so.h, 64, UBF if bf16 else 0.0)
            assert np.all(np.abs(G_st - G_o) <= tol)
            assert np.all(np.abs(G_ctx - G_o) <= tol)
            assert np.all(np.abs(G_st - G_ctx) <= 2 * tol)
        assert np.array_equal(G_st, G_st.T)


def test_gram_static_rejects_sizes_beyond_its_scratch():
    import torch
    import paper_1510_07230_amd as pk
    U = torch.zeros((129, 10, 10, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(pk.PouError):
        pk.gram_static(U, 1.0)
    U = torch.zeros((4, 10, 10, 10), dtype=torch.float64, device="cuda")
    with pytest.raises(pk.PouError):
        pk.gram_static(U, 1.0, bf16=True)
