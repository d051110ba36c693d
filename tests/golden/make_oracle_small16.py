"""Write oracle_small16.json: the oracle's trajectory on the 16^3 workload.

Calls only the oracle and the seeded input module.  Run from the repository
root:  python tests/golden/make_oracle_small16.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import ks, algm  # noqa: E402


def main():
    cfg = synth.CONFIGS["small16"]
    R, Z, s = synth.atoms(cfg)
    sys_ = ks.System(cfg.n, cfg.L, R, Z, s, synth.occupations(cfg))
    A = algm.AlgorithmM(synth.orbitals(cfg), sys_)
    steps = [dict(l=r.l, s=r.s, accepted=r.accepted, E=r.E, tau_bb=r.tau_bb, tau=r.tau,
                  zz=r.zz, df=r.df, C=r.C, Q=r.Q) for r in A.run(50)]
    out = {"_source": "oracle Algorithm M, 50 steps, workload small16 (16^3, L=10, "
                      "2 atoms Z=2 sigma=0.5, N=2, f=2, seeds 1001/2001), paper constants",
           "steps": steps}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_small16.json")
    json.dump(out, open(path, "w"), indent=1)
    print("wrote", path, "final E", steps[-1]["E"])


if __name__ == "__main__":
    main()
