"""Discrete Kohn-Sham model on a periodic cubic grid (oracle, FP64, CPU).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Model (section 2.1 of the paper, energy functional eq. "energy"):
    E(U) = sum_i f_i <u_i, K u_i> + <rho, V_ext> + 1/2 <rho, V_H> + E_x[rho]
with K = -1/2 Delta_h, rho = sum_i f_i u_i^2 (section 2.1 defines rho without
occupations; here every orbital is doubly occupied, f_i = 2), and the inner
product <a, b> = h^3 sum_g a_g b_g, the discrete form of the L2 product of
section 2.2.

Discretisation (section 2.3 leaves it open): a uniform periodic n^3 grid of
spacing h = L/n, point g = (k n + j) n + i for (x, y, z) = h (i, j, k), and the
standard central 8th-order finite-difference second derivative on each axis.
Arrays are indexed [..., z, y, x] (x fastest).

Potentials:
  * Hartree (the double integral of eq. "energy"; the integral operator of
    H(rho) in section 2.1): on the periodic box with a neutralising background
    V_H = P[rho],  P[f] := 4 pi (-Delta_h)^+ (f - mean f), zero mean.
    The oracle applies P exactly by FFT, since the periodic FD operator is
    diagonal in the discrete Fourier basis.
  * Local pseudopotential (section 2.1, V_loc): each ion is a normalised
    Gaussian charge Z (pi s^2)^(-3/2) exp(-d^2/s^2) whose free-space potential
    is -Z erf(d/s)/d; on the periodic box V_ext = -P[rho_ion] (the
    background-neutralised periodic form).
  * Exchange (section 2.1 eps_xc, LDA as in section 4; exchange only):
    E_x = -C_x h^3 sum rho^(4/3),  v_x = -(3/pi)^(1/3) rho^(1/3),
    C_x = 3/4 (3/pi)^(1/3).
  * Correlation, opt in with TERM_CORR (the LDA of section 4 cites the
    Perdew-Zunger parametrisation): E_c = h^3 sum rho eps_c(r_s), v_c =
    d(rho eps_c)/d rho, spin-unpolarised; see correlation_density().
  * Nonlocal pseudopotential, opt in with TERM_NLOC (section 2.1: the nonlocal
    part V_nloc u = sum_l <xi_l, u> xi_l over projectors xi_l in L^2): here
    four atom-centred Gaussian projectors per ion, one s-type and three p-type,
        xi_s(r) = b_s exp(-d^2 / (2 rc^2)),  xi_a(r) = b_p (d_a / rc) exp(-d^2 / (2 rc^2)),
    d = r - R_I by minimum image, with (rc, b_s, b_p) per ion (System.proj).
    It adds E_nl = sum_i f_i sum_l <xi_l, u_i>^2 to E and V_nloc u_i to H u_i.

Parity: every function here is pinned by CPU tests (closed forms, continuum
limits, brute force, finite differences); see tests/test_oracle_ks.py.
"""
from __future__ import annotations

import dataclasses

import numpy as np

# Central 8th-order second-derivative weights for offsets 0, +-1, +-2, +-3, +-4.
FD8 = (-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0)

TERM_KIN, TERM_EXT, TERM_HARTREE, TERM_XC = 1, 2, 4, 8
TERM_ALL = TERM_KIN | TERM_EXT | TERM_HARTREE | TERM_XC
# LDA correlation (Perdew-Zunger form, spin-unpolarised): opt in, not part of TERM_ALL
TERM_CORR = 16
# nonlocal projectors (section 2.1 V_nloc): opt in, needs System.proj
TERM_NLOC = 32

CX = 0.75 * (3.0 / np.pi) ** (1.0 / 3.0)
VX = (3.0 / np.pi) ** (1.0 / 3.0)


@dataclasses.dataclass
class System:
    n: int
    L: float
    R: np.ndarray          # [M, 3]
    Z: np.ndarray          # [M]
    sigma: np.ndarray      # [M]
    occ: np.ndarray        # [N]
    terms: int = TERM_ALL
    proj: object = None    # [M, 3] (rc, b_s, b_p) per ion for TERM_NLOC, else None

    @property
    def h(self):
        return self.L / self.n

    @property
    def dv(self):
        return self.h ** 3

    @property
    def norb(self):
        return len(self.occ)


# ---------------------------------------------------------------- grid pieces

def laplacian(u, h):
    """Periodic 8th-order FD Laplacian Delta_h over the last three axes.

    Offsets larger than the grid wrap around, so on tiny grids coincident
    neighbours add up (np.roll takes shifts modulo n).
    """
    out = 3.0 * FD8[0] * u
    for m in range(1, 5):
        for ax in (-3, -2, -1):
            out = out + FD8[m] * (np.roll(u, m, axis=ax) + np.roll(u, -m, axis=ax))
    return out / (h * h)


def kinetic(u, h):
    """K u = -1/2 Delta_h u."""
    return -0.5 * laplacian(u, h)


def inner(a, b, h):
    """<a, b> = h^3 sum_g a_g b_g over the last three axes."""
    return h ** 3 * np.sum(a * b, axis=(-3, -2, -1))


def _symbol_1d(n, h):
    """Eigenvalues of -D2 (1-D periodic FD8) on the discrete Fourier modes."""
    theta = 2.0 * np.pi * np.arange(n) / n
    s = FD8[0] + 2.0 * sum(FD8[m] * np.cos(m * theta) for m in range(1, 5))
    return -s / (h * h)


def poisson(f, h):
    """P[f] = 4 pi (-Delta_h)^+ (f - mean f), zero mean, by FFT (exact)."""
    n = f.shape[-1]
    lam1 = _symbol_1d(n, h)
    lam = lam1[:, None, None] + lam1[None, :, None] + lam1[None, None, :]
    F = np.fft.fftn(f, axes=(-3, -2, -1))
    lam = lam.copy()
    lam[0, 0, 0] = 1.0
    V = 4.0 * np.pi * F / lam
    V[..., 0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(V, axes=(-3, -2, -1)))


def grid_offsets(n, L, R):
    """Minimum-image offsets r - R per axis: (dx [n], dy [n], dz [n])."""
    ax = (L / n) * np.arange(n)
    out = []
    for a in range(3):
        d = ax - R[a]
        d = d - L * np.round(d / L)
        out.append(d)
    return out


# ---------------------------------------------------------------- ions

def ion_density(sys: System):
    """rho_ion = sum_I Z_I (pi s_I^2)^(-3/2) exp(-d_I^2 / s_I^2), minimum image."""
    n = sys.n
    rho = np.zeros((n, n, n))
    for I in range(len(sys.Z)):
        dx, dy, dz = grid_offsets(n, sys.L, sys.R[I])
        d2 = dz[:, None, None] ** 2 + dy[None, :, None] ** 2 + dx[None, None, :] ** 2
        s = sys.sigma[I]
        rho += sys.Z[I] * (np.pi * s * s) ** -1.5 * np.exp(-d2 / (s * s))
    return rho


def external_potential(sys: System):
    """V_ext = -P[rho_ion]: periodic, neutralised local pseudopotential."""
    return -poisson(ion_density(sys), sys.h)


def _ion_offsets(sys: System, I):
    n = sys.n
    dx, dy, dz = grid_offsets(n, sys.L, sys.R[I])
    X = np.broadcast_to(dx[None, None, :], (n, n, n))
    Y = np.broadcast_to(dy[None, :, None], (n, n, n))
    Zc = np.broadcast_to(dz[:, None, None], (n, n, n))
    return X, Y, Zc


def projectors(sys: System):
    """The nonlocal projectors xi_l on the grid, [4 M, n, n, n]: for ion I rows
    4I (s-type) and 4I + 1 + a (p-type along axis a = x, y, z)."""
    M = len(sys.Z)
    n = sys.n
    Xi = np.zeros((4 * M, n, n, n))
    for I in range(M):
        rc, bs, bp = sys.proj[I]
        X, Y, Zc = _ion_offsets(sys, I)
        g = np.exp(-(X * X + Y * Y + Zc * Zc) / (2.0 * rc * rc))
        Xi[4 * I] = bs * g
        for a, D in enumerate((X, Y, Zc)):
            Xi[4 * I + 1 + a] = bp * (D / rc) * g
    return Xi


def projector_derivatives(sys: System):
    """d xi_l / d R_{I,a} for the projectors of each ion, [M, 4, 3, n, n, n]
    (the ion position enters through d = r - R_I, so d/dR = -d/dd)."""
    M = len(sys.Z)
    n = sys.n
    out = np.zeros((M, 4, 3, n, n, n))
    for I in range(M):
        rc, bs, bp = sys.proj[I]
        D = _ion_offsets(sys, I)
        g = np.exp(-(D[0] ** 2 + D[1] ** 2 + D[2] ** 2) / (2.0 * rc * rc))
        for a in range(3):
            # d g / d d_a = -(d_a / rc^2) g
            dg = -(D[a] / (rc * rc)) * g
            out[I, 0, a] = -bs * dg
            for b in range(3):
                dxi = bp * (D[b] / rc) * dg + (bp / rc * g if a == b else 0.0)
                out[I, 1 + b, a] = -dxi
    return out


def nonlocal_active(sys: System):
    return bool(sys.terms & TERM_NLOC) and sys.proj is not None and len(sys.Z) > 0


def nonlocal_overlaps(U, Xi, h):
    """C[l, i] = <xi_l, u_i>."""
    P = Xi.shape[0]
    N = U.shape[0]
    return h ** 3 * (Xi.reshape(P, -1) @ U.reshape(N, -1).T)


def nonlocal_apply(U, Xi, h):
    """V_nloc u_i = sum_l <xi_l, u_i> xi_l for every orbital."""
    C = nonlocal_overlaps(U, Xi, h)
    P = Xi.shape[0]
    return (C.T @ Xi.reshape(P, -1)).reshape(U.shape)


def nonlocal_energy(U, Xi, sys: System):
    """E_nl = sum_i f_i <u_i, V_nloc u_i> = sum_i f_i sum_l <xi_l, u_i>^2."""
    C = nonlocal_overlaps(U, Xi, sys.h)
    return float(np.sum(sys.occ[None, :] * C * C))


# ---------------------------------------------------------------- density, XC

def density(U, occ):
    """rho = sum_i f_i u_i^2."""
    return np.einsum("i,i...->...", occ, U * U)


def exchange(rho, h):
    """LDA exchange: (E_x, v_x) for a non-negative density."""
    r13 = np.cbrt(np.maximum(rho, 0.0))
    ex = -CX * h ** 3 * np.sum(r13 * r13 * r13 * r13)
    vx = -VX * r13
    return ex, vx


# Perdew-Zunger fit of the correlation energy per electron of the uniform
# electron gas (spin-unpolarised), the LDA of section 4 (ref. PeZu):
#   r_s >= 1:  eps_c = G / (1 + B1 sqrt(r_s) + B2 r_s)
#   r_s <  1:  eps_c = A ln r_s + B + C r_s ln r_s + D r_s
# with r_s = (3 / (4 pi rho))^(1/3); the potential is d(rho eps_c)/d rho =
# eps_c - (r_s / 3) d eps_c / d r_s.
PZ_G, PZ_B1, PZ_B2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116


def correlation_density(rho):
    """(eps_c, v_c) pointwise; both vanish where rho <= 0."""
    rho = np.asarray(rho, dtype=np.float64)
    pos = rho > 0.0
    rs = np.where(pos, np.cbrt(3.0 / (4.0 * np.pi * np.where(pos, rho, 1.0))), 1.0)
    sq = np.sqrt(rs)
    den = 1.0 + PZ_B1 * sq + PZ_B2 * rs
    eps_hi = PZ_G / den
    # -(r_s/3) d eps/d r_s = eps * (B1 sqrt(r_s)/2 + B2 r_s) / (3 den)
    v_hi = eps_hi + eps_hi * (0.5 * PZ_B1 * sq + PZ_B2 * rs) / (3.0 * den)
    lr = np.log(rs)
    eps_lo = PZ_A * lr + PZ_B + PZ_C * rs * lr + PZ_D * rs
    # d eps/d r_s = A / r_s + C (ln r_s + 1) + D
    v_lo = eps_lo - (PZ_A + PZ_C * rs * (lr + 1.0) + PZ_D * rs) / 3.0
    eps = np.where(rs >= 1.0, eps_hi, eps_lo)
    v = np.where(rs >= 1.0, v_hi, v_lo)
    return np.where(pos, eps, 0.0), np.where(pos, v, 0.0)


def correlation(rho, h):
    """LDA correlation: (E_c, v_c) = (h^3 sum rho eps_c, d(rho eps_c)/d rho)."""
    eps, v = correlation_density(rho)
    return float(h ** 3 * np.sum(np.maximum(rho, 0.0) * eps)), v


# ---------------------------------------------------------------- energy, H

@dataclasses.dataclass
class EnergyTerms:
    E: float
    E_kin: float
    E_ext: float
    E_H: float
    E_x: float
    E_c: float = 0.0
    E_nl: float = 0.0


def potentials(U, sys: System, vext=None):
    """(rho, V_H, v_xc, V_eff, E_x, V_ext, E_c) for orbitals U [N, n, n, n]."""
    h = sys.h
    rho = density(U, sys.occ)
    zeros = np.zeros_like(rho)
    VH = poisson(rho, h) if sys.terms & TERM_HARTREE else zeros
    if sys.terms & TERM_XC:
        ex, vx = exchange(rho, h)
    else:
        ex, vx = 0.0, zeros
    ec = 0.0
    if sys.terms & TERM_CORR:
        ec, vc = correlation(rho, h)
        vx = vx + vc
    if vext is None:
        vext = external_potential(sys) if sys.terms & TERM_EXT else zeros
    veff = vx + VH + vext
    if not sys.terms & TERM_EXT:
        veff = vx + VH
    return rho, VH, vx, veff, ex, vext, ec


def energy(U, sys: System, vext=None) -> EnergyTerms:
    """Total energy, eq. "energy" of section 2.1, on the grid."""
    h = sys.h
    rho, VH, vx, veff, ex, vext, ec = potentials(U, sys, vext)
    ekin = 0.0
    if sys.terms & TERM_KIN:
        ekin = float(np.sum(sys.occ * inner(U, kinetic(U, h), h)))
    eext = float(inner(rho, vext, h)) if sys.terms & TERM_EXT else 0.0
    eh = float(0.5 * inner(rho, VH, h)) if sys.terms & TERM_HARTREE else 0.0
    enl = nonlocal_energy(U, projectors(sys), sys) if nonlocal_active(sys) else 0.0
    E = ekin + eext + eh + ex + ec + enl
    return EnergyTerms(E, ekin, eext, eh, float(ex), float(ec), enl)


def hamiltonian_apply(U, sys: System, vext=None):
    """H(rho) u_i = K u_i + V_eff u_i (+ V_nloc u_i)  (section 2.1), rho from U itself."""
    _, _, _, veff, _, _, _ = potentials(U, sys, vext)
    out = veff[None] * U
    if sys.terms & TERM_KIN:
        out = out + kinetic(U, sys.h)
    if nonlocal_active(sys):
        out = out + nonlocal_apply(U, projectors(sys), sys.h)
    return out


def hamiltonian_apply_fixed(U, veff, h, kin=True, Xi=None):
    """H u for a given V_eff (no density recomputation); Xi: projectors of
    the nonlocal term, if any."""
    out = veff[None] * U
    if kin:
        out = out + kinetic(U, h)
    if Xi is not None:
        out = out + nonlocal_apply(U, Xi, h)
    return out


def energy_gradient(U, sys: System, vext=None):
    """Exact gradient of the discrete E w.r.t. the array U: 2 f_i h^3 (H u_i).

    Section 2.1 writes E_{u_i} = H(rho) u_i, leaving out the factor 2 f_i that
    the occupation-weighted energy carries, and the h^3 of the grid sum.
    """
    HU = hamiltonian_apply(U, sys, vext)
    return 2.0 * sys.occ[:, None, None, None] * sys.dv * HU


def forces(U, sys: System):
    """(dE/dR [M,3], dE/dsigma [M]) at fixed U.

    E depends on the ions only through E_ext = <rho, V_ext> = -<P[rho], rho_ion>
    (P is symmetric in <.,.>), so dE/dq = -<V_H, d rho_ion / dq> with V_H = P[rho].
    """
    h, n = sys.h, sys.n
    rho = density(U, sys.occ)
    VH = poisson(rho, h)
    M = len(sys.Z)
    dR = np.zeros((M, 3))
    ds = np.zeros(M)
    for I in range(M):
        dx, dy, dz = grid_offsets(n, sys.L, sys.R[I])
        X = np.broadcast_to(dx[None, None, :], (n, n, n))
        Y = np.broadcast_to(dy[None, :, None], (n, n, n))
        Zc = np.broadcast_to(dz[:, None, None], (n, n, n))
        d2 = X * X + Y * Y + Zc * Zc
        s = sys.sigma[I]
        g = sys.Z[I] * (np.pi * s * s) ** -1.5 * np.exp(-d2 / (s * s))
        # d rho_I / d R_a = g * 2 (r - R)_a / s^2
        for a, D in enumerate((X, Y, Zc)):
            dR[I, a] = -inner(VH, g * 2.0 * D / (s * s), h)
        # d rho_I / d s = g * (2 d^2 / s^3 - 3 / s)
        ds[I] = -inner(VH, g * (2.0 * d2 / s ** 3 - 3.0 / s), h)
    if nonlocal_active(sys):
        # dE_nl / dR_Ia = sum_i f_i sum_{l of I} 2 <xi_l, u_i> <d xi_l / dR_Ia, u_i>
        Xi = projectors(sys)
        C = nonlocal_overlaps(U, Xi, h)
        dXi = projector_derivatives(sys)
        for I in range(M):
            for a in range(3):
                Cd = nonlocal_overlaps(U, dXi[I, :, a], h)  # [4, N]
                dR[I, a] += float(np.sum(sys.occ[None, :] * 2.0 * C[4 * I:4 * I + 4] * Cd))
    return dR, ds


def orth_error(W, h):
    """max |<W^T W> - I|."""
    N = W.shape[0]
    Wf = W.reshape(N, -1)
    G = h ** 3 * (Wf @ Wf.T)
    return float(np.max(np.abs(G - np.eye(N))))


def energy_and_h(U, sys: System, vext=None):
    """(EnergyTerms, H U, sigma_ii = <u_i, H u_i>) from one set of potentials."""
    h = sys.h
    rho, VH, vx, veff, ex, vext, ec = potentials(U, sys, vext)
    KU = kinetic(U, h) if sys.terms & TERM_KIN else np.zeros_like(U)
    ekin = float(np.sum(sys.occ * inner(U, KU, h)))
    eext = float(inner(rho, vext, h)) if sys.terms & TERM_EXT else 0.0
    eh = float(0.5 * inner(rho, VH, h)) if sys.terms & TERM_HARTREE else 0.0
    HU = KU + veff[None] * U
    enl = 0.0
    if nonlocal_active(sys):
        Xi = projectors(sys)
        HU = HU + nonlocal_apply(U, Xi, h)
        enl = nonlocal_energy(U, Xi, sys)
    terms = EnergyTerms(ekin + eext + eh + ex + ec + enl, ekin, eext, eh, float(ex), float(ec),
                        enl)
    sigma = inner(U, HU, h)
    return terms, HU, sigma
