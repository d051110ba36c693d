"""Single steps of the mixed form against the oracle from the same state
(shared by the small-grid and full-size parity tests).

The oracle is handed the GPU's own iterates (as FP64), so trajectory drift
does not enter: per step the backtracking exponent s must be equal, tau_BB
within the bound that the FP32 directions allow, the new block element-wise
within the bound of the FP32 trial point plus its measured distance from
orthonormality, and the reported energy equal to the oracle's energy of the
GPU's block to the bound of the FP32 kinetic sums (tests/_common.py)."""
import numpy as np
import pytest

import synth
from oracle import ks, orth as oorth, algm
from _common import (oracle_system, gpu_system, to_np, kinetic_energy_tolerance,
                     hamiltonian_error_bound, U32, LAM)


def _f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _oracle_from_state(so, p, W, Wp, C, Q, l, E):
    """Algorithm M positioned at iteration l with iterate W and previous iterate
    Wp (both as handed over by the GPU), C, Q and E of the GPU's last step."""
    A = algm.AlgorithmM(W, so, p, orthonormalize_start=False)
    if Wp is not None:
        _, HWp, sigp = ks.energy_and_h(Wp, so, A.vext)
        A.Wp = Wp
        A.Zp = HWp - sigp[:, None, None, None] * Wp
    A.l, A.C, A.Q, A.E = l, C, Q, E
    return A


def _bb_tolerance(W, Wp, so, A, dZ, dZp):
    """Relative bound on tau_BB from FP32 directions: S = W - Wp is formed from
    the same FP32 values (one rounding), Y = Z - Zp carries the direction
    errors dZ + dZp per element; each trace is off by LAM sqrt(sum (a db)^2)."""
    h3 = so.h ** 3
    S = W - Wp
    Y = A.direction() - A.Zp
    dY = dZ + dZp
    dS = U32 * np.abs(S)
    ss = h3 * np.sum(S * S)
    sy = abs(h3 * np.sum(S * Y))
    yy = h3 * np.sum(Y * Y)
    e_ss = 2 * LAM * h3 * np.sqrt(np.sum((S * dS) ** 2))
    e_sy = LAM * h3 * (np.sqrt(np.sum((S * dY) ** 2)) + np.sqrt(np.sum((Y * dS) ** 2)))
    e_yy = 2 * LAM * h3 * np.sqrt(np.sum((Y * dY) ** 2))
    tau1 = e_ss / ss + e_sy / sy
    tau2 = e_sy / sy + e_yy / yy
    return tau1 if (A.l % 2 == 1) else tau2


def _direction_error(W, so, vext):
    rho, VH, vx, veff, ex, _, _ = ks.potentials(W, so, vext)
    _, HW, sig = ks.energy_and_h(W, so, vext)
    dH = hamiltonian_error_bound(W, veff, so.h)
    ng = W[0].size
    dsig = LAM * np.sqrt(ng) * U32 * np.abs(sig)
    return dH + dsig[:, None, None, None] * np.abs(W) + 2 * U32 * np.abs(HW)


def step_parity(cfg, steps, label, proj=None):
    so = oracle_system(cfg, proj=proj)
    p = algm.Params()
    p.tau_init = 1.0 / algm.lambda_max_kinetic(so.h)
    W0 = _f32(oorth.orth(synth.orbitals(cfg), so.h)[0])
    g = gpu_system(cfg, "mixed", proj=proj, tau_init=p.tau_init)
    U = g.new_block(W0)
    vext = ks.external_potential(so)
    prev, cur = None, W0
    last = None
    cache = {}

    def derr(W):
        key = id(W)
        if key not in cache:
            cache[key] = _direction_error(W, so, vext)
        return cache[key]
    for k in range(steps):
        if last is None:
            A = algm.AlgorithmM(cur, so, p, orthonormalize_start=False)
        else:
            A = _oracle_from_state(so, p, cur, prev, last["C"], last["Q"], k, last["E"])
        info = g.step_(U)
        Wg = to_np(U).astype(np.float64)
        if prev is not None:
            btol = _bb_tolerance(cur, prev, so, A, derr(cur), derr(prev))
        r = A.step()
        # the new block against the oracle's, from the same state
        Gg = oorth.gram(Wg, so.h)
        dev = float(np.max(np.abs(Gg - np.eye(cfg.norb))))
        colsum = np.max(np.sum(np.abs(A.W.reshape(cfg.norb, -1)), axis=0))
        dWt = derr(cur) * r.tau + 3 * U32 * np.abs(cur)
        tolU = 2.0 * float(np.max(dWt)) + 2.0 * dev * colsum + 2 * U32 * np.max(np.abs(A.W))
        dU = float(np.max(np.abs(Wg - A.W)))
        # the GPU's energy of its own new block against the oracle's energy of it
        E_o = ks.energy(Wg, so, vext).E
        tolE = kinetic_energy_tolerance(Wg, so.occ, so.h) + 1e-10 * abs(E_o)
        msg = (f"[{label}] step {k}: s {info['s']}/{r.s} tau_bb {info['tau_bb']:.10e}/"
               f"{r.tau_bb:.10e} |dU| {dU:.2e} (tol {tolU:.2e}) E {info['E']:.10f} "
               f"E_oracle(U) {E_o:.10f} (tol {tolE:.2e}) orth {dev:.1e}")
        print(msg, flush=True)
        assert info["s"] == r.s, msg
        if prev is None:
            assert info["tau_bb"] == pytest.approx(r.tau_bb, rel=1e-15)
        else:
            assert abs(info["tau_bb"] - r.tau_bb) <= btol * r.tau_bb, (msg, btol)
        assert dU <= tolU, msg
        assert abs(info["E"] - E_o) <= tolE, msg
        if prev is not None:
            cache.pop(id(prev), None)
        prev, cur, last = cur, Wg, info
    return g, U


