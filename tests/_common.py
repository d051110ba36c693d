"""Helpers shared by the GPU parity tests: build matching oracle and library
systems from the same seeded inputs."""
import numpy as np

import synth
from oracle import ks


def oracle_system(cfg, terms=ks.TERM_ALL):
    R, Z, s = synth.atoms(cfg)
    return ks.System(cfg.n, cfg.L, R, Z, s, synth.occupations(cfg), terms)


def gpu_system(cfg, precision="fp64", **params):
    import paper_1510_07230_amd as pk
    R, Z, s = synth.atoms(cfg)
    p = pk.default_params(**params)
    return pk.System(cfg.n, cfg.L, R, Z, s, synth.occupations(cfg), precision=precision,
                     params=p)


def to_np(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / max(1e-300, np.max(np.abs(b))))
