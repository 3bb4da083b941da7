"""Adjoint sections of the generated plan against directional derivatives of the oracle.

The residual is a polynomial of degree two in T and in B and linear in f, so a
central difference (g(p + h v) - g(p - h v)) / (2h) equals the directional
derivative up to rounding.  The dot-product test <x, J v> = <J^T x, v> then
checks the plan's vector-Jacobian products (run with the numpy interpreter) against
derivatives of the oracle alone, for random x and v.
"""
import os

import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R
from tests.plan_numpy import Interpreter, prepare

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PLAN = os.path.join(ROOT, "paper_2511_03567_amd", "plan.txt")
H = 1e-3


@pytest.fixture(scope="module")
def plan_text():
    with open(PLAN) as fh:
        return fh.read()


def _sym2(rng, nH, nP, m2, scale=1.0):
    x = rng.standard_normal((nH, nH, nP, nP)) * scale
    return 0.5 * (x + x.transpose(1, 0, 3, 2)) * m2


def _setup(nc, na, nv, naux, seed):
    cfg = S.custom_config("adj", nc, na, nv, naux, seed)
    inp = S.make_inputs(cfg)
    nH, nP = nc + na, na + nv
    rng = np.random.default_rng(seed + 100)
    m1, m2 = R.block_mask(nc, na, nv)
    T1 = rng.standard_normal((nH, nP)) * 0.05 * m1
    T2 = _sym2(rng, nH, nP, m2, 0.05)
    x1 = rng.standard_normal((nH, nP)) * m1
    x2 = _sym2(rng, nH, nP, m2)
    v1 = rng.standard_normal((nH, nP)) * m1
    v2 = _sym2(rng, nH, nP, m2)
    n = nc + na + nv
    df = rng.standard_normal((n, n))
    df = df + df.T
    dB = rng.standard_normal((naux, n, n))
    dB = dB + dB.transpose(0, 2, 1)
    return cfg, inp, (T1, T2), (x1, x2), (v1, v2), df, dB


def _run(plan_text, section, cfg, inp, T, x=None, B=None, f=None):
    nc, na, nv, naux = cfg.nc, cfg.na, cfg.nv, cfg.naux
    nH, nP = nc + na, na + nv
    n = nc + na + nv
    B = inp.B if B is None else B
    f = inp.f if f is None else f
    tens = prepare(f, B, inp.G1, inp.G2, inp.G3, nc, na, nv)
    tens.update(T1=T[0], T2=T[1], dT1=np.zeros((nH, nP)), dT2=np.zeros((nH, nH, nP, nP)),
                dF=np.zeros((n, n)), dB=np.zeros((naux, n, n)))
    if x is not None:
        tens.update(XR1=x[0], XL=x[1])
    Interpreter(plan_text, nc, na, nv, naux).run(section, tens)
    return tens


def _dot(a, b):
    return float(sum(np.sum(p * q) for p, q in zip(a, b)))


CASES = [(2, 4, 10, 48, 1), (1, 2, 3, 7, 2), (3, 0, 6, 11, 3), (0, 3, 4, 9, 4)]


@pytest.mark.parametrize("nc,na,nv,naux,seed", CASES)
def test_residual_vjp_amplitudes(plan_text, nc, na, nv, naux, seed):
    cfg, inp, T, x, v, _, _ = _setup(nc, na, nv, naux, seed)
    ref = R.Reference(nc, na, nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
    rp = ref.residual(T[0] + H * v[0], T[1] + H * v[1])
    rm = ref.residual(T[0] - H * v[0], T[1] - H * v[1])
    jv = [(a - b) / (2 * H) for a, b in zip(rp, rm)]
    out = _run(plan_text, "adjoint_t", cfg, inp, T, x)
    want = _dot(x, jv)
    got = _dot((out["dT1"], out["dT2"]), v)
    assert abs(got - want) <= 1e-9 * abs(want)
    d2 = out["dT2"]
    assert np.array_equal(d2, d2.transpose(1, 0, 3, 2))


@pytest.mark.parametrize("nc,na,nv,naux,seed", CASES)
def test_residual_vjp_fock_and_df(plan_text, nc, na, nv, naux, seed):
    cfg, inp, T, x, _, df, dB = _setup(nc, na, nv, naux, seed)
    out = _run(plan_text, "adjoint_theta", cfg, inp, T, x)
    G = (inp.G1, inp.G2, inp.G3)
    rf = [R.Reference(nc, na, nv, inp.f + sg * H * df, inp.B, *G).residual(*T) for sg in (1, -1)]
    rb = [R.Reference(nc, na, nv, inp.f, inp.B + sg * H * dB, *G).residual(*T) for sg in (1, -1)]
    jf = [(a - b) / (2 * H) for a, b in zip(*rf)]
    jb = [(a - b) / (2 * H) for a, b in zip(*rb)]
    for want, got in ((_dot(x, jf), float(np.sum(out["dF"] * df))), (_dot(x, jb), float(np.sum(out["dB"] * dB)))):
        assert abs(got - want) <= 1e-9 * abs(want)


@pytest.mark.parametrize("nc,na,nv,naux,seed", CASES)
def test_energy_gradient(plan_text, nc, na, nv, naux, seed):
    cfg, inp, T, _, v, df, dB = _setup(nc, na, nv, naux, seed)
    G = (inp.G1, inp.G2, inp.G3)
    out = _run(plan_text, "energy_grad", cfg, inp, T)
    ref = R.Reference(nc, na, nv, inp.f, inp.B, *G)
    et = (ref.energy(T[0] + H * v[0], T[1] + H * v[1]) - ref.energy(T[0] - H * v[0], T[1] - H * v[1])) / (2 * H)
    ef = (R.Reference(nc, na, nv, inp.f + H * df, inp.B, *G).energy(*T)
          - R.Reference(nc, na, nv, inp.f - H * df, inp.B, *G).energy(*T)) / (2 * H)
    eb = (R.Reference(nc, na, nv, inp.f, inp.B + H * dB, *G).energy(*T)
          - R.Reference(nc, na, nv, inp.f, inp.B - H * dB, *G).energy(*T)) / (2 * H)
    got = [_dot((out["dT1"], out["dT2"]), v), float(np.sum(out["dF"] * df)), float(np.sum(out["dB"] * dB))]
    for g, w in zip(got, (et, ef, eb)):
        assert abs(g - w) <= 1e-9 * abs(w)
