"""Pins of the oracle's two-fold commutator terms with active orbitals (Section 2.2).

The oracle builds the quadratic residual from the generalized-Wick expansion (Section 2.1)
of [X, T] with X = [H, T], keeping a pair (x, t) unless both amplitudes carry an active
index, and then dropping the terms with a two-body cumulant and the terms of rank > 2.

1. With T = T_ext + T_act (T_act: the amplitude blocks with an active index), the pairs the
   oracle keeps sum to [[H,T],T] - [[H,T_act],T_act].  On a multi-determinant reference
   (1 core, CAS(2,2), 1 virtual orbital: 8 spin orbitals) the engine's expansion of those
   pairs at every rank, lambda_2 and lambda_3 contractions included, must equal the exact
   operator (HTT - 2THT + TTH) - (H Ta Ta - 2 Ta H Ta + Ta Ta H) on random Fock-space vectors.
   No four-body cumulant can arise here (one amplitude has no active leg), and the engine
   generates none, so this equality is exact.
2. The residual's term list (Section 2.2 approximations, reading R1) is that pinned list cut
   by two predicates on its terms: rank 1 or 2, and no lambda_2 factor.  Checked exactly,
   term by term, on the canonical merged forms.
3. The pair filter is itself a predicate on the terms: the expansion of every pair minus the
   terms whose two amplitude factors both carry an active index is the pinned list.
4. A rank-3 operator (legs in every space) commuted with a rank-2 amplitude block, the
   [X_3, T_2] products the quadratic terms are built from, equals the brute-force commutator.
"""
import itertools

import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R
from oracle import wick as W
from oracle.wick import A, C, G, V, Term
from tests.fockspace import Fock, GNO, embed_reference

NC, NA, NV = 1, 2, 1
N = NC + NA + NV
NSO = 2 * N

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def small():
    rng = np.random.default_rng(23)
    F = Fock(NSO)
    dets = S.cas_determinants(NA)
    cvec = rng.standard_normal(dets.size)
    psi = embed_reference(F, NC, NA, N, dets, cvec)
    gno = GNO(F, psi)
    sp = R.Spaces(NC, NA, NV)
    aso = sp.so[A]
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
    assert np.abs(l2).max() > 1e-2 and np.abs(l3).max() > 1e-2     # a genuinely correlated reference
    base = {"g1": (g1, (aso, aso)), "e1": (np.eye(m) - g1, (aso, aso)),
            "l2": (l2, (aso,) * 4), "l3": (l3, (aso,) * 6)}
    return F, gno, sp, base, rng


def _engine_coefficients(terms, ev, sp):
    """Coefficient arrays over every spin-orbital index, by rank, of a list of terms."""
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


def _hamiltonian_and_amplitudes(sp, rng):
    """Random spin-orbital f, DF factors, and amplitudes on the blocks of the cluster operator."""
    n = N
    f = rng.standard_normal((n, n))
    f = f + f.T
    B = S.make_df(rng, n, 3)
    fso = np.zeros((NSO, NSO))
    fso[:n, :n] = fso[n:, n:] = f
    Bso = np.zeros((3, NSO, NSO))
    Bso[:, :n, :n] = Bso[:, n:, n:] = B
    # <pq||rs> = (pr|qs) - (ps|qr) over spin orbitals
    v = np.einsum("Xpr,Xqs->pqrs", Bso, Bso) - np.einsum("Xps,Xqr->pqrs", Bso, Bso)
    t1 = np.zeros((NSO, NSO))
    for sk, sc in R.T1_BLOCKS:
        t1[np.ix_(sp.so[sk], sp.so[sc])] = rng.standard_normal((len(sp.so[sk]), len(sp.so[sc])))
    t2 = np.zeros((NSO,) * 4)
    for blk in R.T2_BLOCKS:
        idx = [sp.so[s] for s in blk]
        t2[np.ix_(*idx)] += rng.standard_normal([len(i) for i in idx])
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    # each ordered block holds the antisymmetrized values: keep them only on the stored blocks
    mask = np.zeros((NSO,) * 4, dtype=bool)
    for blk in R.T2_BLOCKS:
        mask[np.ix_(*[sp.so[s] for s in blk])] = True
    t2 = t2 * mask
    return fso, Bso, v, t1 * 0.3, t2 * 0.3


def _active_mask(sp, rank):
    act = np.zeros(NSO, dtype=bool)
    act[sp.so[A]] = True
    if rank == 1:
        return act[:, None] | act[None, :]
    return act[:, None, None, None] | act[None, :, None, None] | act[None, None, :, None] | act[None, None, None, :]


@pytest.fixture(scope="module")
def quadratic(small):
    F, gno, sp, base, rng = small
    fso, Bso, v, t1, t2 = _hamiltonian_and_amplitudes(sp, rng)
    full = list(range(NSO))
    tens = dict(base)
    tens.update({"f": (fso, (full, full)), "B": (Bso, (None, full, full)),
                 "t1": (t1, (full, full)), "t2": (t2, (full,) * 4)})
    ev = R.Evaluator(sp, tens)
    Hs, Ts = R.hamiltonian_terms(), R.cluster_terms()
    X = W.merge(W.commutator(Hs, Ts))

    def keep(x, t):
        return not (R._has_active_amp(x) and R._has_active_amp(t))

    Q = W.merge(W.commutator(X, Ts, pair_filter=keep))
    return F, gno, sp, ev, (fso, v, t1, t2), X, Ts, Q


def test_kept_pairs_equal_double_commutator_minus_active_active(quadratic):
    F, gno, sp, ev, (fso, v, t1, t2), X, Ts, Q = quadratic
    assert any(n == "l2" for t in Q for n, _ in t.factors)
    assert any(n == "l3" for t in Q for n, _ in t.factors)
    assert max(t.rank for t in Q) == 4
    eng = _engine_coefficients(Q, ev, sp)
    ma1, ma2 = _active_mask(sp, 1), _active_mask(sp, 2)
    # operators in the strings' coefficient convention: {a^c_k} t1[k,c], 1/4 {a^{cd}_{kl}} t2[k,l,c,d]
    Hc = {1: fso, 2: 0.25 * v}
    Tc = {1: t1.T.copy(), 2: 0.25 * np.einsum("klcd->cdkl", t2)}
    Ac = {1: (t1 * ma1).T.copy(), 2: 0.25 * np.einsum("klcd->cdkl", t2 * ma2)}
    for trial in range(2):
        y = np.random.default_rng(100 + trial).standard_normal(F.dim)
        vid = ("quad", trial)
        ap = lambda co, x, tag: gno.operator_apply(co, x, vid + tag)
        Ty = ap(Tc, y, ("T",))
        Hy = ap(Hc, y, ("H",))
        HTy = ap(Hc, Ty, ("HT",))
        full = ap(Hc, ap(Tc, Ty, ("TT",)), ("HTT",)) - 2 * ap(Tc, HTy, ("THT",)) + ap(Tc, ap(Tc, Hy, ("TH",)), ("TTH",))
        Ay = ap(Ac, y, ("A",))
        HAy = ap(Hc, Ay, ("HA",))
        act = ap(Hc, ap(Ac, Ay, ("AA",)), ("HAA",)) - 2 * ap(Ac, HAy, ("AHA",)) + ap(Ac, ap(Ac, Hy, ("AH",)), ("AAH",))
        want = full - act
        got = ap(eng, y, ("eng",))
        assert np.abs(want).max() > 1e-3
        assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()
    gno._vec_cache.clear()


def _canon(terms):
    acc = {}
    for t in terms:
        key, sg = W.canonical(t)
        acc[key] = acc.get(key, 0) + t.coef * sg
    return {k: c for k, c in acc.items() if c != 0}


def test_residual_terms_are_the_pinned_list_cut_by_rank_and_lambda2(quadratic):
    _, _, _, _, _, X, Ts, Q = quadratic
    cut = [t for t in Q if t.rank in (1, 2) and not any(n == "l2" for n, _ in t.factors)]
    assert len(cut) < len(Q)
    kept = R.term_lists()["quad_R"]
    assert _canon(cut) == _canon(kept)


def test_pair_filter_is_a_predicate_on_amplitude_factors(quadratic):
    _, _, _, _, _, X, Ts, Q = quadratic
    every = W.merge(W.commutator(X, Ts))

    def both_active(t):
        counts = R.amplitude_active_counts(t)
        return len(counts) == 2 and all(c > 0 for c in counts)

    dropped = [t for t in every if both_active(t)]
    assert dropped
    assert _canon([t for t in every if not both_active(t)]) == _canon(Q)


def test_rank3_with_rank2_amplitude_matches_fock_space(small):
    F, gno, sp, base, rng = small
    ra, rb = 3, 2
    sa, sb = (G,) * 6, (A, V, C, A)          # t^{cd}_{kl}: upper (A, V), lower (C, A)
    Ta = np.zeros((NSO,) * 6)
    Ta[np.ix_(*[sp.so[s] for s in sa])] = rng.standard_normal((NSO,) * 6)
    Tb = np.zeros((NSO,) * 4)
    idx = [sp.so[s] for s in sb]
    Tb[np.ix_(*idx)] = rng.standard_normal([len(i) for i in idx])
    full = list(range(NSO))
    tens = dict(base)
    tens["opA"] = (Ta, (full,) * 6)
    tens["opB"] = (Tb, (full,) * 4)
    ev = R.Evaluator(sp, tens)

    def op(name, rank, spaces):
        labs = list(range(2 * rank))
        seq = [(W.CRE, l) for l in labs[:rank]] + [(W.ANN, l) for l in labs[rank:][::-1]]
        return Term(1, [(name, tuple(labs))], seq, dict(zip(labs, spaces)))

    terms = W.commutator([op("opA", ra, sa)], [op("opB", rb, sb)])
    assert max(t.rank for t in terms) == 4
    assert any(n == "l3" for t in terms for n, _ in t.factors)
    eng = _engine_coefficients(terms, ev, sp)
    y = np.random.default_rng(7).standard_normal(F.dim)
    vid = ("r3r2",)
    got = gno.operator_apply(eng, y, vid)
    By = gno.operator_apply({rb: Tb}, y, vid)
    Ay = gno.operator_apply({ra: Ta}, y, vid)
    want = gno.operator_apply({ra: Ta}, By, vid + ("B",)) - gno.operator_apply({rb: Tb}, Ay, vid + ("A",))
    assert np.abs(want).max() > 1e-3
    assert np.abs(got - want).max() < 1e-10 * np.abs(want).max()
    gno._vec_cache.clear()
