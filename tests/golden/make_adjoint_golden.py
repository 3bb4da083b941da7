"""Writes adjoint_vjp_*.npz: vector-Jacobian products of the oracle's residual, element by element.

Calls only the oracle and the seeded input generators.  For each shape, with seeded amplitudes
T and cotangent x (pair-symmetric, excluded blocks zero) the products are directional derivatives
of f = <x, r(T; f, B)>, taken by central differences.  The residual (Section 2.2) is a polynomial
of degree two in T and B and linear in f, so a central difference is its derivative exactly, up
to rounding.
  dT:  every stored amplitude, along e_j + (its pair image) for T2 (so the stored value is twice
       the pair-symmetric projection unless the element is its own image);
  dF:  f[p][q] and f[q][p] together, p <= q (every pair);
  dB:  B[X][p][q] and B[X][q][p] together, p <= q: every element at the small shape, a seeded
       sample at the larger one.
Run from the repository root (worker processes, one BLAS thread each):
    python tests/golden/make_adjoint_golden.py [workers]
"""
import os
import sys
import time
from multiprocessing import Pool

os.environ.setdefault("OMP_NUM_THREADS", "1")
os.environ.setdefault("OPENBLAS_NUM_THREADS", "1")

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synthetic as S  # noqa: E402
from oracle import ricmrcc as R  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
H = 1e-3
# (nc, na, nv, naux, seed, number of sampled dB elements or None for all)
SHAPES = [(1, 2, 3, 7, 2, None), (2, 4, 10, 48, 1, 100)]


def case_inputs(nc, na, nv, naux, seed):
    """Inputs, amplitudes and cotangent of one shape (the GPU test draws the same ones)."""
    cfg = S.custom_config("adjvjp", nc, na, nv, naux, seed)
    inp = S.make_inputs(cfg)
    nH, nP = nc + na, na + nv
    rng = np.random.default_rng(seed + 300)
    m1, m2 = R.block_mask(nc, na, nv)

    def sym(scale):
        y = rng.standard_normal((nH, nH, nP, nP)) * scale
        return 0.5 * (y + y.transpose(1, 0, 3, 2)) * m2

    T = (rng.standard_normal((nH, nP)) * 0.05 * m1, sym(0.05))
    x = (rng.standard_normal((nH, nP)) * m1, sym(1.0))
    return cfg, inp, T, x


_W = {}


def _init(nc, na, nv, naux, seed):
    cfg, inp, T, x = case_inputs(nc, na, nv, naux, seed)
    _W.update(nc=nc, na=na, nv=nv, inp=inp, T=T, x=x)
    R.term_lists()
    _W["base"] = R.Reference(nc, na, nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)


def _f(f, B, T1, T2):
    w = _W
    if f is w["inp"].f and B is w["inp"].B:
        ref = w["base"]
    else:
        ref = R.Reference(w["nc"], w["na"], w["nv"], f, B, w["inp"].G1, w["inp"].G2, w["inp"].G3)
    r1, r2 = ref.residual(T1, T2)
    return float(np.sum(w["x"][0] * r1) + np.sum(w["x"][1] * r2))


def _job(job):
    kind, idx = job
    w = _W
    f, B = w["inp"].f, w["inp"].B
    T1, T2 = w["T"]
    if kind == "t1":
        E = np.zeros_like(T1)
        E[idx] = 1.0
        return (_f(f, B, T1 + H * E, T2) - _f(f, B, T1 - H * E, T2)) / (2 * H)
    if kind == "t2":
        k, l, c, d = idx
        E = np.zeros_like(T2)
        E[k, l, c, d] = 1.0
        E[l, k, d, c] = 1.0
        return (_f(f, B, T1, T2 + H * E) - _f(f, B, T1, T2 - H * E)) / (2 * H)
    if kind == "f":
        p, q = idx
        E = np.zeros_like(f)
        E[p, q] = 1.0
        E[q, p] = 1.0
        return (_f(f + H * E, B, T1, T2) - _f(f - H * E, B, T1, T2)) / (2 * H)
    X, p, q = idx
    E = np.zeros_like(B)
    E[X, p, q] = 1.0
    E[X, q, p] = 1.0
    return (_f(f, B + H * E, T1, T2) - _f(f, B - H * E, T1, T2)) / (2 * H)


def main():
    workers = int(sys.argv[1]) if len(sys.argv) > 1 else 4
    for nc, na, nv, naux, seed, nsample in SHAPES:
        cfg, inp, T, x = case_inputs(nc, na, nv, naux, seed)
        nH, nP, n = nc + na, na + nv, nc + na + nv
        m1, m2 = R.block_mask(nc, na, nv)
        t1_idx = [tuple(int(v) for v in i) for i in np.argwhere(m1)]
        t2_idx = [(k, l, c, d) for k, l, c, d in (tuple(int(v) for v in i) for i in np.argwhere(m2))
                  if (k, l, c, d) <= (l, k, d, c)]
        f_idx = [(p, q) for p in range(n) for q in range(p, n)]
        b_all = [(X, p, q) for X in range(naux) for p in range(n) for q in range(p, n)]
        if nsample is None:
            b_idx = b_all
        else:
            sel = np.random.default_rng(seed + 400).choice(len(b_all), size=nsample, replace=False)
            b_idx = [b_all[i] for i in sorted(sel)]
        jobs = ([("t1", i) for i in t1_idx] + [("t2", i) for i in t2_idx] + [("f", i) for i in f_idx]
                + [("b", i) for i in b_idx])
        print(f"shape nc={nc} na={na} nv={nv} naux={naux}: {len(jobs)} directional derivatives", flush=True)
        t0 = time.perf_counter()
        vals = []
        with Pool(workers, initializer=_init, initargs=(nc, na, nv, naux, seed)) as pool:
            for i, v in enumerate(pool.imap(_job, jobs, chunksize=8)):
                vals.append(v)
                if (i + 1) % 500 == 0:
                    print(f"  {i + 1} done, {time.perf_counter() - t0:.0f} s", flush=True)
        a, b = len(t1_idx), len(t1_idx) + len(t2_idx)
        c = b + len(f_idx)
        out = os.path.join(HERE, f"adjoint_vjp_{nc}_{na}_{nv}_{naux}.npz")
        np.savez_compressed(
            out, h=H, seed=seed,
            t1_idx=np.array(t1_idx, dtype=np.int64).reshape(-1, 2), t1=np.array(vals[:a]),
            t2_idx=np.array(t2_idx, dtype=np.int64).reshape(-1, 4), t2=np.array(vals[a:b]),
            f_idx=np.array(f_idx, dtype=np.int64).reshape(-1, 2), f=np.array(vals[b:c]),
            b_idx=np.array(b_idx, dtype=np.int64).reshape(-1, 3), b=np.array(vals[c:]))
        print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    main()
