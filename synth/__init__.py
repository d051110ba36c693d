"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module draws random numbers and lays them out; it computes nothing of the
method itself (no stencil, potential, energy, density or orthonormalisation).
Both the CPU oracle and the HIP path receive the arrays produced here and
nothing else in common.

The paper's molecules (benzene ... C1419H556, section 4) need geometries and
Troullier-Martins pseudopotentials that are not available, so synthetic
periodic systems of Gaussian ions stand in for them; their grid sizes (4,096 to
2.1M points) and orbital counts (2 to 512) span the paper's Table 1 range
(Ng 102,705-1,903,841; N 15-3,116).

Recipe (all FP64, numpy PCG64):
  * atoms: positions uniform in [0, L)^3 with seed 1000+cfg; where a minimum
    separation is set, positions are drawn by rejection so that every
    minimum-image pair distance is at least that value;
  * charges Z and Gaussian widths sigma as listed per configuration (the
    differentiation case draws Z from {1, 2, 4} and sigma from U[0.4, 0.7]);
  * nonlocal projector parameters (opt in), seed 3000+cfg: per ion a width
    rc ~ U[0.45, 0.6] bohr and amplitudes b_s ~ U[1, 2], b_p ~ U[0.5, 1.5] of
    one s-type and three p-type Gaussian projectors (stand-ins for the
    Troullier-Martins nonlocal channels of section 4);
  * orbitals, seed 2000+cfg: either i.i.d. N(0, 1) values on the grid, or an
    atom-centred start  u_i = sum_I sum_b c_{iIb} phi_b(r - R_I) exp(-d^2/2)
    with phi_b in {1, dx, dy, dz} and c ~ N(0, 1), a stand-in for the paper's
    LCAO start (section 4).  Four functions per atom keep the block full rank
    whenever N <= 4M.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np


@dataclasses.dataclass(frozen=True)
class Config:
    name: str
    n: int                 # grid points per axis
    L: float               # periodic box side (bohr)
    natoms: int
    Z: object              # float, or tuple of choices drawn uniformly
    sigma: object          # float, or (lo, hi) drawn uniformly
    norb: int
    occ: float = 2.0
    min_sep: Optional[float] = None
    start: str = "random"  # "random" | "atomic"
    cfg_id: int = 0

    @property
    def ng(self) -> int:
        return self.n ** 3

    @property
    def h(self) -> float:
        return self.L / self.n


# The five workloads.  Names say what they are.
CONFIGS = {
    "small16": Config("small16", 16, 10.0, 2, 2.0, 0.5, 2, cfg_id=1),
    "fp64_48": Config("fp64_48", 48, 16.0, 16, 2.0, 0.5, 16, min_sep=1.5, cfg_id=2),
    "grad64": Config("grad64", 64, 20.0, 32, (1.0, 2.0, 4.0), (0.4, 0.7), 32,
                     min_sep=1.5, cfg_id=3),
    "mixed96": Config("mixed96", 96, 24.0, 64, 4.0, 0.5, 128, min_sep=1.5,
                      start="atomic", cfg_id=4),
    "mixed128": Config("mixed128", 128, 32.0, 256, 4.0, 0.5, 512, min_sep=1.5,
                       start="atomic", cfg_id=5),
}


def custom(name, n, L, natoms, Z, sigma, norb, occ=2.0, min_sep=None,
           start="random", seed_id=99) -> Config:
    """A configuration outside the five named workloads (tests, edge cases)."""
    return Config(name, n, L, natoms, Z, sigma, norb, occ, min_sep, start, seed_id)


def _min_image_dist2(a, b, L):
    d = a - b
    d -= L * np.round(d / L)
    return float(np.sum(d * d))


def atoms(cfg: Config):
    """Return (R [M,3], Z [M], sigma [M]) as float64 arrays, seeded by 1000+cfg_id."""
    rng = np.random.default_rng(1000 + cfg.cfg_id)
    M = cfg.natoms
    R = np.zeros((M, 3))
    k = 0
    tries = 0
    while k < M:
        p = rng.uniform(0.0, cfg.L, size=3)
        tries += 1
        if cfg.min_sep is not None:
            if any(_min_image_dist2(p, R[j], cfg.L) < cfg.min_sep ** 2 for j in range(k)):
                if tries > 10_000_000:
                    raise RuntimeError("cannot place atoms with the requested separation")
                continue
        R[k] = p
        k += 1
    if isinstance(cfg.Z, tuple):
        Z = rng.choice(np.array(cfg.Z, dtype=np.float64), size=M)
    else:
        Z = np.full(M, float(cfg.Z))
    if isinstance(cfg.sigma, tuple):
        sig = rng.uniform(cfg.sigma[0], cfg.sigma[1], size=M)
    else:
        sig = np.full(M, float(cfg.sigma))
    return R, Z, sig


def occupations(cfg: Config):
    return np.full(cfg.norb, float(cfg.occ))


def orbitals(cfg: Config, dtype=np.float64, variant=0):
    """Raw (not orthonormal) start block, shape [N, n, n, n] (z, y, x; x fastest).
    variant > 0 draws another start of the same kind (other coefficients)."""
    rng = np.random.default_rng(2000 + cfg.cfg_id + 7919 * variant)
    n, N = cfg.n, cfg.norb
    if cfg.start == "random":
        U = rng.standard_normal((N, n, n, n))
        return U.astype(dtype, copy=False)
    R, _, _ = atoms(cfg)
    M = R.shape[0]
    if N > 4 * M:
        raise ValueError("atomic start needs N <= 4 * natoms")
    C = rng.standard_normal((N, M, 4)).reshape(N, 4 * M)
    U = np.empty((N, n, n, n), dtype=dtype)
    ax = cfg.h * np.arange(n)

    def axis_offsets(a):
        d = ax[None, :] - R[:, a][:, None]          # [M, n]
        return d - cfg.L * np.round(d / cfg.L)

    dxs, dys, dzs = axis_offsets(0), axis_offsets(1), axis_offsets(2)
    zchunk = max(1, int(2_000_000 // (4 * M * n * n)) or 1)
    for z0 in range(0, n, zchunk):
        z1 = min(n, z0 + zchunk)
        dz = dzs[:, z0:z1][:, :, None, None]
        dy = dys[:, None, :, None]
        dx = dxs[:, None, None, :]
        g = np.exp(-0.5 * (dx * dx + dy * dy + dz * dz))   # [M, nz, n, n]
        B = np.stack([g, g * dx, g * dy, g * dz], axis=1)  # [M, 4, nz, n, n]
        B = B.reshape(4 * M, -1)
        U[:, z0:z1] = (C @ B).reshape(N, z1 - z0, n, n).astype(dtype, copy=False)
    return U


def projector_params(cfg: Config, rc=(0.45, 0.6), b_s=(1.0, 2.0), b_p=(0.5, 1.5)):
    """Per-ion parameters (rc, b_s, b_p) of the synthetic nonlocal projectors,
    [M, 3], drawn uniformly from the given ranges with seed 3000+cfg."""
    rng = np.random.default_rng(3000 + cfg.cfg_id)
    M = cfg.natoms
    return np.stack([rng.uniform(*rc, size=M), rng.uniform(*b_s, size=M),
                     rng.uniform(*b_p, size=M)], axis=1)


def random_direction(shape, seed):
    """Seeded N(0,1) array used for finite-difference directions in tests."""
    return np.random.default_rng(seed).standard_normal(shape)
