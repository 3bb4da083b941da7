"""Writes oracle_solve.json: converged energies of the CPU oracle's regularized iteration.

Calls only the oracle and the seeded input generators.  Run from the repository root:
    python tests/golden/make_solve_golden.py            # every case
    python tests/golden/make_solve_golden.py --diis [name ...]   # (some of) the DIIS cases, merged by name

"cases": the oracle's plain regularized Jacobi iteration (eq. ric-update) from T = 0.
"diis_cases": the same fixed point reached faster by DIIS over the oracle's update, for shapes
where the plain iteration takes too long on the CPU: the CAS(8,8) active space (full 3-body
RDM of 4900 determinants) with the core of the CAS(8,8) workload and 40 virtual orbitals.  The
workload's own 120 virtuals are out of reach: the oracle's spin-orbital vvvv block alone is
26.5 GB there, and one residual does not fit in 64 GB.
The extrapolation below only mixes the oracle's own updates U(T_i) with weights that minimize
|sum c_i (U(T_i) - T_i)| under sum c_i = 1; the stored energy is taken after a plain oracle
step whose length is below the tolerance, so it is a fixed point of the oracle's update.
"""
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synthetic as S  # noqa: E402
from oracle import ricmrcc as R  # noqa: E402

CASES = [("tiny_cas44", 0.5), ("tiny_cas44", 0.25)]
TOL = 1e-10
# (name, nc, na, nv, naux, seed, s): the CAS(8,8) active space on 40 virtuals, and the CAS(6,6)
# workload of the adjoint tests (nc=6, nv=60, naux=180) whole
DIIS_CASES = [("cas88_nv40", 10, 8, 40, 120, 2, 0.5), ("adjoint_cas66", 6, 6, 60, 180, 3, 0.5)]
DIIS_TOL = 1e-9
DIIS_M = 6


def solve_diis(ref, s, tol, m, max_iter=100):
    """DIIS over the oracle's regularized update; returns (E_corr, iterations, last step)."""
    sp = ref.sp
    D1, D2 = R.denominators(ref.f, sp.nc, sp.na, sp.nv)
    m1, m2 = R.block_mask(sp.nc, sp.na, sp.nv)
    T1 = np.zeros((sp.nH, sp.nP))
    T2 = np.zeros((sp.nH, sp.nH, sp.nP, sp.nP))
    hist = []
    for it in range(1, max_iter + 1):
        t0 = time.perf_counter()
        R1, R2 = ref.residual(T1, T2)
        N1 = R.ric_update(T1, R1, D1, s) * m1
        N2 = R.ric_update(T2, R2, D2, s) * m2
        e1, e2 = N1 - T1, N2 - T2
        step = math.sqrt(float(np.sum(e1 * e1) + np.sum(e2 * e2)))
        print(f"  it {it}: step {step:.3e} ({time.perf_counter() - t0:.0f} s)", flush=True)
        if step < tol:
            return ref.energy(N1, N2), it, step
        hist.append((N1, N2, e1, e2))
        hist = hist[-m:]
        k = len(hist)
        A = np.zeros((k + 1, k + 1))
        for i in range(k):
            for j in range(i + 1):
                A[i, j] = A[j, i] = float(np.sum(hist[i][2] * hist[j][2]) + np.sum(hist[i][3] * hist[j][3]))
        A[k, :k] = A[:k, k] = -1.0
        rhs = np.zeros(k + 1)
        rhs[k] = -1.0
        c = np.linalg.lstsq(A, rhs, rcond=None)[0][:k]
        T1 = sum(ci * h[0] for ci, h in zip(c, hist))
        T2 = sum(ci * h[1] for ci, h in zip(c, hist))
    raise RuntimeError("DIIS did not converge")


def main():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_solve.json")
    if "--diis" in sys.argv:
        names = sys.argv[sys.argv.index("--diis") + 1:] or [c[0] for c in DIIS_CASES]
        with open(path) as fh:
            doc = json.load(fh)
        new = {c["config"]: c for c in run_diis(names)}
        old = [c for c in doc.get("diis_cases", []) if c["config"] not in new]
        doc["diis_cases"] = old + list(new.values())
        with open(path, "w") as fh:
            json.dump(doc, fh, indent=1)
        return
    doc = {"source": "oracle.ricmrcc.solve (regularized Jacobi from T = 0, eq. ric-update)",
           "cases": run_plain(), "diis_cases": run_diis()}
    with open(path, "w") as fh:
        json.dump(doc, fh, indent=1)


def run_diis(names=None):
    out = []
    for name, nc, na, nv, naux, seed, s in DIIS_CASES:
        if names is not None and name not in names:
            continue
        cfg = S.custom_config(name, nc, na, nv, naux, seed)
        inp = S.make_inputs(cfg)
        ref = R.Reference(cfg.nc, cfg.na, cfg.nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
        print(f"{name} s={s}: DIIS({DIIS_M}) over the oracle's update", flush=True)
        e, it, step = solve_diis(ref, s, DIIS_TOL, DIIS_M)
        out.append({"config": name, "nc": nc, "na": na, "nv": nv, "naux": naux, "seed": seed, "s": s,
                    "tol": DIIS_TOL, "diis": DIIS_M, "e_corr": e, "e0": ref.reference_energy(),
                    "iterations": it, "last_step": step})
        print(out[-1], flush=True)
    return out


def run_plain():
    out = []
    for name, s in CASES:
        cfg = S.CONFIGS[name]
        inp = S.make_inputs(cfg)
        ref = R.Reference(cfg.nc, cfg.na, cfg.nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
        e, _, _, it = R.solve(ref, s, tol=TOL)
        out.append({"config": name, "s": s, "tol": TOL, "e_corr": e, "e0": ref.reference_energy(),
                    "iterations": it})
        print(out[-1], flush=True)
    return out


if __name__ == "__main__":
    main()
