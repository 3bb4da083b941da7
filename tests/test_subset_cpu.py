"""Exactness of the orbital-subset reduction that the full-size GPU check samples with.

Oracle on both sides: the residuals and energy of the whole problem, with amplitudes
that vanish outside chosen core and virtual orbitals, against those of the problem
restricted to (chosen cores + all actives + chosen virtuals).
"""
import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R

import orbital_subset as OS


@pytest.mark.parametrize("nc,na,nv,naux,cores,virts", [
    (5, 4, 13, 40, [0, 2, 4], [0, 5, 6, 12]),
    (4, 3, 11, 30, [3], [1, 10]),
    (3, 0, 12, 30, [0, 2], [4, 7, 11]),
])
def test_subset_residual_and_energy_exact(nc, na, nv, naux, cores, virts):
    cfg = S.custom_config("subset", nc, na, nv, naux, 31)
    inp = S.make_inputs(cfg)
    ncs, nvs = len(cores), len(virts)
    fs, Bs = OS.restrict(inp.f, inp.B, nc, na, cores, virts)
    rng = np.random.default_rng(5)
    m1, m2 = R.block_mask(ncs, na, nvs)
    T1s = rng.standard_normal((ncs + na, na + nvs)) * 0.05 * m1
    T2s = rng.standard_normal((ncs + na,) * 2 + (na + nvs,) * 2) * 0.05
    T2s = 0.5 * (T2s + T2s.transpose(1, 0, 3, 2)) * m2
    hm, pm = OS.hole_map(nc, na, cores), OS.particle_map(na, virts)
    T1, T2 = OS.embed(T1s, T2s, hm, pm, nc + na, na + nv)

    full = R.Reference(nc, na, nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
    sub = R.Reference(ncs, na, nvs, fs, Bs, inp.G1, inp.G2, inp.G3)
    R1, R2 = full.residual(T1, T2)
    R1s, R2s = sub.residual(T1s, T2s)
    R1f, R2f = full.residual(np.zeros_like(T1), np.zeros_like(T2))
    d2 = R2[np.ix_(hm, hm, pm, pm)] - R2f[np.ix_(hm, hm, pm, pm)]
    assert np.abs(d2).max() > 1e-3                       # the amplitudes matter on the subset
    assert np.abs(R1[np.ix_(hm, pm)] - R1s).max() < 1e-13
    assert np.abs(R2[np.ix_(hm, hm, pm, pm)] - R2s).max() < 1e-13
    e, es = full.energy(T1, T2), sub.energy(T1s, T2s)
    assert abs(e) > 1e-4
    assert abs(e - es) < 1e-13
