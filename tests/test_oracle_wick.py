"""Pins of the oracle's generalized-Wick engine against brute-force Fock-space algebra.

For random operators A (legs in every space) and B (legs restricted to one
amplitude block), the engine's expansion of [A, B] into generalized
normal-ordered strings, with contractions gamma, eta, lambda_2, lambda_3 of a
multi-determinant reference (Section 2.1), must reproduce the exact operator
A B - B A applied to random vectors.
"""
import itertools

import numpy as np
import pytest

from oracle import ricmrcc as R
from oracle import wick as W
from oracle.wick import A, C, G, V, Term
from tests.fockspace import Fock, GNO

NC, NA, NV = 1, 3, 1
N = NC + NA + NV
NSO = 2 * N


def _active_glob(t, s):
    return s * N + NC + t


@pytest.fixture(scope="module")
def system():
    rng = np.random.default_rng(11)
    F = Fock(NSO)
    core = [0, N]
    psi = np.zeros(F.dim)
    import synthetic as S
    dets = S.cas_determinants(NA)
    cvec = rng.standard_normal(dets.size)
    for d, c in zip(dets, cvec):
        occ = list(core)
        for s in (0, 1):
            for t in range(NA):
                if (int(d) >> (t + s * NA)) & 1:
                    occ.append(_active_glob(t, s))
        psi += c * F.basis_vector(occ)
    psi /= np.linalg.norm(psi)
    gno = GNO(F, psi)
    aso = [_active_glob(t, s) for s in (0, 1) for t in range(NA)]
    m = len(aso)
    g1 = np.array([[gno.rdm([p], [q]) for q in aso] for p in aso])
    g2 = np.zeros((m,) * 4)
    for i, j, k, l in itertools.product(range(m), repeat=4):
        g2[i, j, k, l] = gno.rdm([aso[i], aso[j]], [aso[k], aso[l]])
    g3 = np.zeros((m,) * 6)
    for idx in itertools.product(range(m), repeat=6):
        if len(set(idx[:3])) == 3 and len(set(idx[3:])) == 3:
            g3[idx] = gno.rdm([aso[i] for i in idx[:3]], [aso[i] for i in idx[3:]])
    l2, l3 = R.spinorbital_cumulants(g1, g2, g3)
    sp = R.Spaces(NC, NA, NV)
    base = {"g1": (g1, (aso, aso)), "e1": (np.eye(m) - g1, (aso, aso)),
            "l2": (l2, (aso,) * 4), "l3": (l3, (aso,) * 6)}
    return F, gno, sp, base, rng


def _op(name, rank, spaces):
    labs = list(range(2 * rank))
    seq = [(W.CRE, l) for l in labs[:rank]] + [(W.ANN, l) for l in labs[rank:][::-1]]
    return Term(1, [(name, tuple(labs))], seq, dict(zip(labs, spaces)))


def _random_tensor(rng, sp, rank, spaces):
    T = np.zeros((NSO,) * (2 * rank))
    idx = [sp.so[s] for s in spaces]
    T[np.ix_(*idx)] = rng.standard_normal([len(i) for i in idx])
    return T


def _engine_operator(terms, ev, sp):
    full = list(range(NSO))
    coeffs = {}
    for t in terms:
        r = t.rank
        U, L = t.upper(), t.lower()
        outs = [t.space[l] for l in U + L]
        val = ev.term(t, U + L, outs)
        if r not in coeffs:
            coeffs[r] = np.zeros((NSO,) * (2 * r)) if r else 0.0
        if r == 0:
            coeffs[r] += float(val)
        else:
            R._scatter(sp, coeffs[r], (full,) * (2 * r), val, outs)
    return coeffs


CASES = [
    (1, (G, G), 1, (V, A)),
    (2, (G, G, G, G), 1, (A, C)),
    (2, (G, G, G, G), 2, (A, V, A, C)),      # t^{cd}_{kl}: upper (A,V), lower (C,A) -> spaces of labels (c,d,k,l)
    (2, (G, G, G, G), 2, (A, A, A, C)),
    (2, (G, G, G, G), 2, (V, A, A, A)),
    (1, (G, G), 2, (A, A, C, A)),
    (3, (G,) * 6, 1, (A, A)),
    (2, (G, G, G, G), 2, (G, G, G, G)),
]


@pytest.mark.parametrize("ra,sa,rb,sb", CASES)
def test_commutator_matches_fock_space(system, ra, sa, rb, sb):
    F, gno, sp, base, rng = system
    Ta = _random_tensor(rng, sp, ra, sa)
    Tb = _random_tensor(rng, sp, rb, sb)
    full = list(range(NSO))
    tens = dict(base)
    tens["opA"] = (Ta, (full,) * (2 * ra))
    tens["opB"] = (Tb, (full,) * (2 * rb))
    ev = R.Evaluator(sp, tens)
    terms = W.commutator([_op("opA", ra, sa)], [_op("opB", rb, sb)])
    eng = _engine_operator(terms, ev, sp)
    for trial in range(2):
        y = rng.standard_normal(F.dim)
        vid = ("y", ra, rb, sa, sb, trial)
        got = gno.operator_apply(eng, y, vid)
        By = gno.operator_apply({rb: Tb}, y, vid)
        Ay = gno.operator_apply({ra: Ta}, y, vid)
        ABy = gno.operator_apply({ra: Ta}, By, vid + ("B",))
        BAy = gno.operator_apply({rb: Tb}, Ay, vid + ("A",))
        want = ABy - BAy
        assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()
    gno._vec_cache.clear()


def test_merge_preserves_operator(system):
    """Canonical merging of equal terms (tensor antisymmetry, renaming) keeps the sum."""
    F, gno, sp, base, rng = system
    Tv = np.zeros((NSO,) * 4)
    x = rng.standard_normal((NSO,) * 4)
    Tv = x - x.transpose(1, 0, 2, 3) - x.transpose(0, 1, 3, 2) + x.transpose(1, 0, 3, 2)
    Tt = _random_tensor(rng, sp, 2, (C, A, A, V))       # t2 labels (k,l,c,d)
    Tt = Tt - Tt.transpose(1, 0, 2, 3)
    Tt = Tt - Tt.transpose(0, 1, 3, 2)
    full = list(range(NSO))
    ev_tens = dict(base)
    ev_tens["vv"] = (Tv, (full,) * 4)
    ev_tens["t2"] = (Tt, (full,) * 4)
    v = Term(W.Fraction(1, 4), [("vv", (0, 1, 2, 3))],
             [(W.CRE, 0), (W.CRE, 1), (W.ANN, 3), (W.ANN, 2)], {0: G, 1: G, 2: G, 3: G})
    t = Term(W.Fraction(1, 4), [("t2", (0, 1, 2, 3))],
             [(W.CRE, 2), (W.CRE, 3), (W.ANN, 1), (W.ANN, 0)], {0: C, 1: A, 2: A, 3: V})
    W.ANTISYM["vv"] = ((0, 1), (2, 3))
    raw = W.commutator([v], [t])
    merged = W.merge(raw)
    assert len(merged) < len(raw)
    ev = R.Evaluator(sp, ev_tens)
    a = _engine_operator(raw, ev, sp)
    b = _engine_operator(merged, ev, sp)
    from tests.fockspace import antisymmetrize
    for r in a:
        if r == 0:
            assert abs(a[r] - b.get(r, 0.0)) < 1e-12
        else:
            assert np.allclose(antisymmetrize(a[r]), antisymmetrize(b[r]), atol=1e-12)
