"""Spin-multiplet references (Section 2.3.2): the spin-free RDMs of every M_S component of a
multiplet are the same, so the spin-free equations need no change; the generated plan still
equals the oracle for a triplet reference."""
import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R
from tests.plan_numpy import Interpreter, prepare

import os
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PLAN = os.path.join(ROOT, "paper_2511_03567_amd", "plan.txt")


@pytest.mark.parametrize("na", [2, 4])
def test_spinfree_rdms_are_the_same_for_every_ms_component(na):
    rng = np.random.default_rng(40 + na)
    (d1, c1), (d0, c0) = S.random_triplet(rng, na)
    # the M_S = 0 partner is a triplet too: <S^2> = 2
    dets0 = S.cas_determinants(na)
    full = np.zeros(dets0.size)
    pos = {int(d): i for i, d in enumerate(dets0)}
    for d, c in zip(d0, c0):
        full[pos[int(d)]] = c
    assert abs(full @ S._s2_matrix(dets0, na) @ full - 2.0) < 1e-12
    for a, b in zip(S.spinfree_rdms(d1, c1, na, 3), S.spinfree_rdms(d0, c0, na, 3)):
        assert np.abs(a - b).max() < 1e-12


def test_plan_matches_oracle_for_a_triplet_reference():
    nc, na, nv, naux = 2, 4, 6, 20
    cfg = S.custom_config("t", nc, na, nv, naux, 44)
    inp = S.make_inputs(cfg, with_rdms=False)
    (d1, c1), _ = S.random_triplet(np.random.default_rng(45), na)
    G1, G2, G3 = S.spinfree_rdms(d1, c1, na, 3)
    ref = R.Reference(nc, na, nv, inp.f, inp.B, G1, G2, G3)
    nH, nP = nc + na, na + nv
    rng = np.random.default_rng(46)
    m1, m2 = R.block_mask(nc, na, nv)
    T1 = rng.standard_normal((nH, nP)) * 0.05 * m1
    T2 = rng.standard_normal((nH, nH, nP, nP)) * 0.05
    T2 = 0.5 * (T2 + T2.transpose(1, 0, 3, 2)) * m2
    tens = prepare(inp.f, inp.B, G1, G2, G3, nc, na, nv)
    tens.update(T1=T1, T2=T2, R1=np.zeros((nH, nP)), R2=np.zeros((nH, nH, nP, nP)))
    with open(PLAN) as fh:
        it = Interpreter(fh.read(), nc, na, nv, naux)
    it.run("residual", tens)
    it.run("energy", tens)
    r1, r2 = ref.residual(T1, T2)
    assert np.abs(tens["R1"] - r1).max() < 1e-12
    assert np.abs(tens["R2"] - r2).max() < 1e-12
    assert abs(float(tens["E"]) - ref.energy(T1, T2)) < 1e-12
