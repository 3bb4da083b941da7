"""Writes oracle_solve.json: converged energies of the CPU oracle's regularized iteration.

Calls only the oracle and the seeded input generators.  Run from the repository root:
    python tests/golden/make_solve_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synthetic as S  # noqa: E402
from oracle import ricmrcc as R  # noqa: E402

CASES = [("tiny_cas44", 0.5), ("tiny_cas44", 0.25)]
TOL = 1e-10


def main():
    out = []
    for name, s in CASES:
        cfg = S.CONFIGS[name]
        inp = S.make_inputs(cfg)
        ref = R.Reference(cfg.nc, cfg.na, cfg.nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
        e, _, _, it = R.solve(ref, s, tol=TOL)
        out.append({"config": name, "s": s, "tol": TOL, "e_corr": e, "e0": ref.reference_energy(),
                    "iterations": it})
        print(out[-1], flush=True)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_solve.json")
    with open(path, "w") as fh:
        json.dump({"source": "oracle.ricmrcc.solve (regularized Jacobi from T = 0, eq. ric-update)",
                   "cases": out}, fh, indent=1)


if __name__ == "__main__":
    main()
