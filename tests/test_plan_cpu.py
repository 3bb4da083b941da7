"""Host-side checks of the library: its generated contraction plan, and its C ABI symbols.

The plan (paper_2511_03567_amd/plan.txt) is produced by the library's own
equation generator; executing it with the numpy reference interpreter must
reproduce the oracle's energy and residuals.  No GPU is used.
"""
import os
import re
import subprocess

import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R
from tests.plan_numpy import Interpreter, prepare

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PLAN = os.path.join(ROOT, "paper_2511_03567_amd", "plan.txt")
HEADER = os.path.join(ROOT, "include", "ricmrcc.h")
LIB = os.path.join(ROOT, "paper_2511_03567_amd", "libricmrcc.so")


@pytest.fixture(scope="module")
def plan_text():
    with open(PLAN) as fh:
        return fh.read()


@pytest.mark.parametrize("nc,na,nv,naux,seed", [(2, 4, 10, 48, 1), (3, 4, 5, 12, 2), (0, 2, 7, 15, 3),
                                                 (4, 0, 9, 20, 4), (1, 6, 4, 11, 5), (3, 3, 0, 10, 6),
                                                 (1, 1, 1, 3, 7)])
def test_plan_matches_oracle(plan_text, nc, na, nv, naux, seed):
    cfg = S.custom_config("p", nc, na, nv, naux, seed)
    inp = S.make_inputs(cfg)
    ref = R.Reference(nc, na, nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
    nH, nP = nc + na, na + nv
    rng = np.random.default_rng(seed)
    m1, m2 = R.block_mask(nc, na, nv)
    T1 = rng.standard_normal((nH, nP)) * 0.05 * m1
    T2 = rng.standard_normal((nH, nH, nP, nP)) * 0.05
    T2 = 0.5 * (T2 + T2.transpose(1, 0, 3, 2)) * m2
    tens = prepare(inp.f, inp.B, inp.G1, inp.G2, inp.G3, nc, na, nv)
    tens.update(T1=T1, T2=T2, R1=np.zeros((nH, nP)), R2=np.zeros((nH, nH, nP, nP)))
    it = Interpreter(plan_text, nc, na, nv, naux)
    it.run("residual", tens)
    it.run("energy", tens)
    r1, r2 = ref.residual(T1, T2)
    assert np.abs(tens["R1"] - r1).max() < 1e-12
    assert np.abs(tens["R2"] - r2).max() < 1e-12
    assert abs(float(tens["E"]) - ref.energy(T1, T2)) < 1e-12


@pytest.mark.parametrize("nc,na,nv,naux,seed", [(2, 4, 10, 48, 1), (1, 6, 4, 11, 5), (4, 0, 9, 20, 4)])
def test_plan_term_groups_match_oracle_groups(plan_text, nc, na, nv, naux, seed):
    """The plan's residual_lin and residual_quad sections (the term groups ric_residual can select)
    reproduce the oracle's linear and quadratic groups, and add up to the whole residual."""
    cfg = S.custom_config("p", nc, na, nv, naux, seed)
    inp = S.make_inputs(cfg)
    ref = R.Reference(nc, na, nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
    nH, nP = nc + na, na + nv
    rng = np.random.default_rng(seed + 50)
    m1, m2 = R.block_mask(nc, na, nv)
    T1 = rng.standard_normal((nH, nP)) * 0.05 * m1
    T2 = rng.standard_normal((nH, nH, nP, nP)) * 0.05
    T2 = 0.5 * (T2 + T2.transpose(1, 0, 3, 2)) * m2
    it = Interpreter(plan_text, nc, na, nv, naux)
    out = {}
    for sec, grp in (("residual_lin", "lin"), ("residual_quad", "quad"), ("residual", None)):
        tens = prepare(inp.f, inp.B, inp.G1, inp.G2, inp.G3, nc, na, nv)
        tens.update(T1=T1, T2=T2, R1=np.zeros((nH, nP)), R2=np.zeros((nH, nH, nP, nP)))
        it.run(sec, tens)
        out[sec] = (tens["R1"].copy(), tens["R2"].copy())
        if grp is not None:
            r1, r2 = ref.residual(T1, T2, groups=(grp,))
            assert np.abs(out[sec][0] - r1).max() < 1e-12
            assert np.abs(out[sec][1] - r2).max() < 1e-12
    for i in range(2):
        assert np.abs(out["residual_lin"][i] + out["residual_quad"][i] - out["residual"][i]).max() < 1e-12


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.skip("library not built")
    with open(HEADER) as fh:
        declared = set(re.findall(r"^\s*(?:int|void|const char\*)\s+(ric_\w+)\s*\(", fh.read(), re.M))
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r"\sT\s(ric_\w+)", out))
    assert declared and declared <= exported, declared - exported
