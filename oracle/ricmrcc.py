"""Spin-free RIC-MRCCSD energy, many-body residuals and regularized update: CPU oracle.

TEST INFRASTRUCTURE.  Plain, slow, obviously correct; float64 throughout.  Only
tests/, the smoke check and the CPU baseline of the benchmark may use it.

What is computed (the passages of the paper each step follows):

* Hamiltonian in generalized normal order (Section 2.1): H = E0 + f{a^p_q} +
  1/4 v{a^pq_rs}, v^{pq}_{rs} = <pq||rs>, with (pr|qs) = sum_X B[X,p,r] B[X,q,s].
* Cluster operator (Section 2.2): T1 + T2, hole -> particle, every block whose
  indices are all active left out.
* Effective Hamiltonian truncated after the two-fold commutator,
  Hbar = H + [H,T] + 1/2 [[H,T],T] (BCH truncation of Section 2.2).
* Approximations of Section 2.2 on the two-fold commutator (reading R1):
    energy:    drop a term when both of its amplitudes carry three active indices;
    residuals: drop a term when both of its amplitudes carry an active index, and
               drop every term that contains the two-body cumulant.
  Leg counting shows no kept term can hold a four-body cumulant: a fully
  contracted <[[H2,T2],T2]> with x and y active legs on the amplitudes has
  2(x+y)-4 active legs, so lambda_4 needs x = y = 3; residual terms keep at most
  one active amplitude (at most 3 + 4 - 1 active legs).
* Many-body residuals (Section 2.2): E = Hbar_0, r^c_k = Hbar^c_k, r^{cd}_{kl} =
  Hbar^{cd}_{kl}; the two-body part is antisymmetrized as in eq. (antisym) of
  Section 3.1 and only the alpha-beta sector is kept (Section 3.1).
* Spin-free storage (Section 2.3.1, Table 2): T1[k,c] = t^c_k (alpha),
  T2[k,l,c,d] = t^{c dbar}_{k lbar}; T2[k,l,c,d] = T2[l,k,d,c]
  (eq. spinfree-perm-sym).  All other spin blocks follow from the singlet
  relations of Section 2.3.1 and Table 2.
* Spin-orbital RDMs of the reference are built from the spin-free Gamma1..3
  with the all-alpha and partial-trace relations of Section 2.3.1; cumulants
  from them by eq. (cumulant) and its three-body analogue.
* Regularized update (eq. ric-update):
  t <- (t Delta + r) (1 - exp(-s Delta^2)) / Delta, Delta from diag(f) (eq. cc-update).
* Reference energy: E0 = <Psi0|H|Psi0> with h obtained by inverting the
  generalized Fock matrix definition of Section 2.1.

Index conventions: spatial orbitals are ordered core, active, virtual (Table 1);
the hole range H = core + active, the particle range P = active + virtual.
Spin orbitals are numbered sigma*n + p (alpha block, then beta block).
"""
from __future__ import annotations

import itertools
import math
import os
import pickle
from functools import lru_cache

import numpy as np

from . import wick as W
from .wick import A, C, G, H, P, V, Term

# ----------------------------------------------------------------------------------------
# operators


def hamiltonian_terms():
    f = Term(1, [("f", (0, 1))], [(W.CRE, 0), (W.ANN, 1)], {0: G, 1: G})
    v = Term(W.Fraction(1, 4), [("v", (0, 1, 2, 3))],
             [(W.CRE, 0), (W.CRE, 1), (W.ANN, 3), (W.ANN, 2)], {0: G, 1: G, 2: G, 3: G})
    return [f, v]


T1_BLOCKS = [(C, A), (C, V), (A, V)]                       # IT, IA, TA  (TU left out)
T2_BLOCKS = [(sk, sl, sc, sd) for sk in (C, A) for sl in (C, A) for sc in (A, V) for sd in (A, V)
             if not (sk == A and sl == A and sc == A and sd == A)]  # TUVW left out


def cluster_terms():
    out = []
    for sk, sc in T1_BLOCKS:
        out.append(Term(1, [("t1", (0, 1))], [(W.CRE, 1), (W.ANN, 0)], {0: sk, 1: sc}))
    for sk, sl, sc, sd in T2_BLOCKS:
        out.append(Term(W.Fraction(1, 4), [("t2", (0, 1, 2, 3))],
                        [(W.CRE, 2), (W.CRE, 3), (W.ANN, 1), (W.ANN, 0)],
                        {0: sk, 1: sl, 2: sc, 3: sd}))
    return out


def amplitude_active_counts(term):
    """Number of active indices of every amplitude factor of a term."""
    return [sum(1 for l in ls if term.space[l] == A) for n, ls in term.factors if n in ("t1", "t2")]


def _has_active_amp(term):
    return any(c > 0 for c in amplitude_active_counts(term))


def _has_three_active_amp(term):
    return any(c == 3 for c in amplitude_active_counts(term))


@lru_cache(maxsize=None)
def term_lists(variant: str = "R1"):
    """Energy and residual term lists of Hbar (spin-orbital, generalized normal order).

    Returns dict with keys 'lin' (H + [H,T] terms of rank 0..2) and 'quad_E',
    'quad_R' (the filtered two-fold commutator, WITHOUT the factor 1/2).
    The result is cached on disk next to this file (pure function of the code).
    """
    cache = os.path.join(os.path.dirname(__file__), f".terms_{variant}.pkl")
    src_stamp = _source_stamp()
    if os.path.exists(cache):
        try:
            with open(cache, "rb") as fh:
                stamp, data = pickle.load(fh)
            if stamp == src_stamp:
                return data
        except Exception:
            pass
    Hs = hamiltonian_terms()
    Ts = cluster_terms()
    X = W.merge(W.commutator(Hs, Ts, max_rank=3))
    lin = [t for t in Hs + X if t.rank <= 2]

    def res_pair(x, t):
        return not (_has_active_amp(x) and _has_active_amp(t))

    def en_pair(x, t):
        return not (_has_three_active_amp(x) and _has_three_active_amp(t))

    qR = W.commutator(X, Ts, max_rank=2, pair_filter=res_pair)
    qR = [t for t in qR if t.rank in (1, 2) and not any(n == "l2" for n, _ in t.factors)]
    qR = W.merge(qR)
    qE = W.merge(W.commutator(X, Ts, max_rank=0, pair_filter=en_pair))
    data = {"lin": lin, "quad_R": qR, "quad_E": qE}
    try:
        with open(cache, "wb") as fh:
            pickle.dump((src_stamp, data), fh)
    except OSError:
        pass
    return data


def _source_stamp():
    import hashlib
    h = hashlib.sha256()
    d = os.path.dirname(__file__)
    for fn in ("wick.py", "ricmrcc.py"):
        with open(os.path.join(d, fn), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


# ----------------------------------------------------------------------------------------
# spin-orbital tensors from spin-free inputs


def _letters(k):
    return "abcdefghijklmnopqrstuvwxyz"[:k]


def _canonical_blocks(Gs):
    """Canonical spin blocks C_m (m alpha columns first) of a k-body singlet tensor."""
    k = Gs.ndim // 2
    if k == 1:
        return {1: Gs / 2.0, 0: Gs / 2.0}
    if k == 2:
        swap = np.einsum("qprs->pqrs", Gs)
        aa = (Gs - swap) / 6.0                     # all-alpha, Section 2.3.1
        ab = (2.0 * Gs + swap) / 6.0               # alpha-beta via the partial trace
        return {2: aa, 1: ab, 0: aa}
    if k == 3:
        rpq = np.einsum("rpqstu->pqrstu", Gs)      # O^{RPQ}_{STU} at (p,q,r,s,t,u)
        qrp = np.einsum("qrpstu->pqrstu", Gs)
        qpr = np.einsum("qprstu->pqrstu", Gs)
        aaa = (Gs + rpq + qrp) / 12.0              # all-alpha with the permutation sum rule
        aab = (Gs - qpr) / 6.0 - aaa               # partial trace over the third column
        abb = np.einsum("qrptus->pqrstu", aab)     # spin flip of (b a a) then column reorder
        return {3: aaa, 2: aab, 1: abb, 0: aaa}
    raise ValueError(k)


def spinorbital_tensor(Gs):
    """Full antisymmetric spin-orbital tensor (2na)^(2k) of a singlet k-body spin-free tensor.

    Local spin-orbital index sigma*na + t.
    """
    k = Gs.ndim // 2
    na = Gs.shape[0]
    blocks = _canonical_blocks(Gs)
    out = np.zeros((2 * na,) * (2 * k))
    L = _letters(2 * k)
    for su in itertools.product((0, 1), repeat=k):
        for sl in itertools.product((0, 1), repeat=k):
            m = su.count(0)
            if sl.count(0) != m:
                continue
            pu = sorted(range(k), key=lambda i: su[i])
            pl = sorted(range(k), key=lambda i: sl[i])
            sign = W._parity(pu) * W._parity(pl)
            src = "".join(L[i] for i in pu) + "".join(L[k + i] for i in pl)
            blk = sign * np.einsum(src + "->" + L, blocks[m])
            idx = [np.arange(na) + s * na for s in su] + [np.arange(na) + s * na for s in sl]
            out[np.ix_(*idx)] = blk
    return out


def spinorbital_cumulants(g1, g2, g3):
    """lambda2, lambda3 from spin-orbital RDMs (eq. cumulant and its three-body analogue)."""
    l2 = g2 - np.einsum("pr,qs->pqrs", g1, g1) + np.einsum("ps,qr->pqrs", g1, g1)
    l3 = g3.copy()
    up = "pqr"
    lo = "stu"
    for i in range(3):
        for j in range(3):
            ru = up[:i] + up[i + 1:]
            rl = lo[:j] + lo[j + 1:]
            sgn = (-1) ** (i + j)
            l3 -= sgn * np.einsum(f"{up[i]}{lo[j]},{ru}{rl}->pqrstu", g1, l2)
    for perm in itertools.permutations(range(3)):
        sgn = W._parity(list(perm))
        l3 -= sgn * np.einsum(f"p{lo[perm[0]]},q{lo[perm[1]]},r{lo[perm[2]]}->pqrstu", g1, g1, g1)
    return l2, l3


def spinfree_cumulants(G1, G2, G3):
    """Spin-free two- and three-body cumulants from spin-free RDMs.

    Lambda2 = Gamma2 - G1 G1 + 1/2 G1 G1 (exchange): the spin sum of eq. (cumulant).
    Lambda3: the spin sum of the three-body cumulant of a singlet, written with
    Gamma1 and Lambda2 (upper p,q,r paired with lower s,t,u):
      Gamma3 - [G^p_s L^{qr}_{tu} + G^q_t L^{pr}_{su} + G^r_u L^{pq}_{st}]
      + 1/2 [G^p_t L^{qr}_{su} + G^p_u L^{qr}_{ts} + G^q_s L^{pr}_{tu} + G^q_u L^{pr}_{st}
             + G^r_s L^{pq}_{ut} + G^r_t L^{pq}_{su}]
      - G^p_s G^q_t G^r_u + 1/2 [G^p_s G^q_u G^r_t + G^p_t G^q_s G^r_u + G^p_u G^q_t G^r_s]
      - 1/4 [G^p_t G^q_u G^r_s + G^p_u G^q_s G^r_t]
    (the product weights are -sgn(pi) 2^(cycles(pi)-3)).  Both are pinned against
    spin sums of spin-orbital cumulants of S = 0 states in the tests.
    """
    e = np.einsum
    L2 = G2 - e("pr,qs->pqrs", G1, G1) + 0.5 * e("ps,qr->pqrs", G1, G1)
    L3 = (G3
          - (e("ps,qrtu->pqrstu", G1, L2) + e("qt,prsu->pqrstu", G1, L2) + e("ru,pqst->pqrstu", G1, L2))
          + 0.5 * (e("pt,qrsu->pqrstu", G1, L2) + e("pu,qrts->pqrstu", G1, L2)
                   + e("qs,prtu->pqrstu", G1, L2) + e("qu,prst->pqrstu", G1, L2)
                   + e("rs,pqut->pqrstu", G1, L2) + e("rt,pqsu->pqrstu", G1, L2))
          - e("ps,qt,ru->pqrstu", G1, G1, G1)
          + 0.5 * (e("ps,qu,rt->pqrstu", G1, G1, G1) + e("pt,qs,ru->pqrstu", G1, G1, G1)
                   + e("pu,qt,rs->pqrstu", G1, G1, G1))
          - 0.25 * (e("pt,qu,rs->pqrstu", G1, G1, G1) + e("pu,qs,rt->pqrstu", G1, G1, G1)))
    return L2, L3


class Spaces:
    def __init__(self, nc, na, nv):
        self.nc, self.na, self.nv = nc, na, nv
        self.n = n = nc + na + nv
        core = list(range(nc))
        act = list(range(nc, nc + na))
        vir = list(range(nc + na, n))
        so = lambda lst: lst + [n + p for p in lst]
        self.so = {C: so(core), A: so(act), V: so(vir)}
        self.so[H] = self.so[C] + self.so[A]
        self.so[P] = self.so[A] + self.so[V]
        self.so[G] = self.so[C] + self.so[A] + self.so[V]
        self.nH = nc + na
        self.nP = na + nv


def spinorbital_amplitudes(sp: Spaces, T1, T2):
    """Spin-orbital t1 (2n x 2n) and t2 over (H,H,P,P) from spin-free T1[H,P], T2[H,H,P,P]."""
    n, nH, nP = sp.n, sp.nH, sp.nP
    t1 = np.zeros((2 * n, 2 * n))
    Hs, Ps = sp.so[H], sp.so[P]
    for s in (0, 1):
        hi = [s * n + p for p in range(nH)]
        pi = [s * n + sp.nc + q for q in range(nP)]
        t1[np.ix_(hi, pi)] = T1
    # t2 over local (H,H,P,P) spin-orbital ranges: H local = (core a, act a, core b, act b)
    t2 = np.zeros((2 * nH, 2 * nH, 2 * nP, 2 * nP))
    Tx = np.einsum("klcd->kldc", T2)
    for sk, sl, sc, sd in itertools.product((0, 1), repeat=4):
        if sk + sl != sc + sd:
            continue
        if (sk, sl) == (sc, sd) and sk != sl:
            blk = T2                                  # (a b; a b), (b a; b a)
        elif sk != sl and (sk, sl) == (sd, sc):
            blk = -Tx                                 # (a b; b a), (b a; a b)
        elif sk == sl == sc == sd:
            blk = T2 - Tx                             # same spin
        else:
            continue
        idx = (_loc(sk, nH), _loc(sl, nH), _loc(sc, nP), _loc(sd, nP))
        t2[np.ix_(*idx)] = blk
    return t1, t2


def _loc(s, m):
    return np.arange(m) + s * m


# ----------------------------------------------------------------------------------------
# evaluation of term lists


class Evaluator:
    """Evaluates terms with numpy.einsum on spin-orbital tensors (one einsum per term)."""

    def __init__(self, sp: Spaces, tensors: dict):
        # tensors: name -> (array, tuple of axis ranges as lists of global spin-orbitals or None)
        self.sp = sp
        self.tensors = tensors
        self._pos = {}
        self._cache = {}

    def _positions(self, rng_key, rng, space):
        key = (rng_key, space)
        if key not in self._pos:
            where = {g: i for i, g in enumerate(rng)}
            self._pos[key] = np.array([where[g] for g in self.sp.so[space]], dtype=np.int64)
        return self._pos[key]

    def block(self, name, spaces):
        key = (name, spaces)
        if key in self._cache:
            return self._cache[key]
        arr, ranges = self.tensors[name]
        idx = []
        for ax, (rng, s) in enumerate(zip(ranges, spaces)):
            if rng is None:
                idx.append(np.arange(arr.shape[ax]))
            else:
                idx.append(self._positions((name, ax), rng, s))
        blk = arr[np.ix_(*idx)]
        self._cache[key] = blk
        return blk

    def antisym_eri(self, spaces):
        """<pq||rs> = (pr|qs) - (ps|qr) over spin orbitals, for one block of spaces (cached).

        Built a slice of p at a time: each library product then has fewer than 2^31 output
        elements (the limit of 32-bit BLAS indexing), with the same sums over X."""
        key = ("v", spaces)
        if key not in self._cache:
            sp, sq, sr, ss = spaces
            B = lambda a, b: self.block("B", (None, a, b))
            Bpr, Bqs, Bps, Bqr = B(sp, sr), B(sq, ss), B(sp, ss), B(sq, sr)
            npp, nq, nr, ns = Bpr.shape[1], Bqs.shape[1], Bpr.shape[2], Bqs.shape[2]
            v = np.empty((npp, nq, nr, ns))
            step = max(1, (1 << 28) // max(1, nq * nr * ns))
            for p0 in range(0, npp, step):
                sl = slice(p0, p0 + step)
                v[sl] = np.einsum("Xpr,Xqs->pqrs", Bpr[:, sl], Bqs, optimize=True)
                v[sl] -= np.einsum("Xps,Xqr->pqrs", Bps[:, sl], Bqr, optimize=True)
            self._cache[key] = v
        return self._cache[key]

    def term(self, t: Term, out_labels, out_spaces):
        """Value of the term's coefficient tensor over out_labels (each restricted to out_spaces)."""
        space = dict(t.space)
        for l, s in zip(out_labels, out_spaces):
            space[l] &= s
            if not space[l]:
                return None
        letters = {}
        pool = iter("abcdefghijklmnopqrstuvwxyzABCDEFGHIJKLMNOPQRSTUVWXYZ")

        def let(l):
            if l not in letters:
                letters[l] = next(pool)
            return letters[l]

        variants = [[(1.0, [(name, ls)]) for name, ls in t.factors]]
        out = None
        for var in variants:
            coef = float(t.coef)
            ops = []
            subs = []
            aux = 0
            for c, fl in var:
                coef *= c
                for name, ls in fl:
                    if name == "v":
                        ops.append(self.antisym_eri(tuple(space[x] for x in ls)))
                    else:
                        ops.append(self.block(name, tuple(space[x] for x in ls)))
                    subs.append("".join(let(x) for x in ls))
            spec = ",".join(subs) + "->" + "".join(let(l) for l in out_labels)
            val = coef * np.einsum(spec, *ops, optimize="greedy")
            out = val if out is None else out + val
        return out


def _scatter(sp, acc, acc_ranges, val, spaces):
    idx = []
    for rng, s in zip(acc_ranges, spaces):
        where = {g: i for i, g in enumerate(rng)}
        idx.append(np.array([where[g] for g in sp.so[s]], dtype=np.int64))
    acc[np.ix_(*idx)] += val


class Reference:
    """Spin-orbital description of one problem: spaces, f, B, RDMs and cumulants."""

    def __init__(self, nc, na, nv, f, B, G1, G2, G3):
        self.sp = sp = Spaces(nc, na, nv)
        n = sp.n
        self.f, self.B, self.G1, self.G2, self.G3 = f, B, G1, G2, G3
        self.naux = B.shape[0]
        fso = np.zeros((2 * n, 2 * n))
        fso[:n, :n] = f
        fso[n:, n:] = f
        Bso = np.zeros((self.naux, 2 * n, 2 * n))
        Bso[:, :n, :n] = B
        Bso[:, n:, n:] = B
        if na:
            # Section 2.3.2: spin-free cumulants from the spin-free RDMs, then their spin blocks
            L2, L3 = spinfree_cumulants(G1, G2, G3)
            g1 = spinorbital_tensor(G1)
            l2 = spinorbital_tensor(L2)
            l3 = spinorbital_tensor(L3)
            e1 = np.eye(2 * na) - g1
        else:
            g1 = e1 = np.zeros((0, 0))
            l2 = np.zeros((0,) * 4)
            l3 = np.zeros((0,) * 6)
        self.g1, self.l2, self.l3, self.e1 = g1, l2, l3, e1
        Gr, Ar = list(range(2 * n)), sp.so[A]      # f, B, t1 are stored in natural order
        self.base = {
            "f": (fso, (Gr, Gr)),
            "B": (Bso, (None, Gr, Gr)),
            "g1": (g1, (Ar, Ar)),
            "e1": (e1, (Ar, Ar)),
            "l2": (l2, (Ar,) * 4),
            "l3": (l3, (Ar,) * 6),
        }

    # --- reference energy -------------------------------------------------------------
    def eri(self):
        return np.einsum("Xpq,Xrs->pqrs", self.B, self.B)

    def core_hamiltonian(self):
        """h from f by inverting f = h + sum_core v + sum_active v gamma (Section 2.1), spin-free."""
        sp = self.sp
        nc, na = sp.nc, sp.na
        Bc = self.B[:, :nc, :nc]
        J = np.einsum("Xpq,Xii->pq", self.B, Bc)
        K = np.einsum("Xpi,Xiq->pq", self.B[:, :, :nc], self.B[:, :nc, :])
        Ba = self.B[:, nc:nc + na, nc:nc + na]
        Ja = np.einsum("Xpq,Xtu,tu->pq", self.B, Ba, self.G1)
        Ka = np.einsum("Xpu,Xtq,tu->pq", self.B[:, :, nc:nc + na], self.B[:, nc:nc + na, :], self.G1)
        return self.f - (2 * J - K) - (Ja - 0.5 * Ka)

    def reference_energy(self):
        """E0 = sum h D1 + 1/2 sum (pq|rs) D2^{pr}_{qs}, full-space spin-free RDMs."""
        sp = self.sp
        nc, na = sp.nc, sp.na
        m = nc + na
        D1 = np.zeros((m, m))
        D1[:nc, :nc] = 2 * np.eye(nc)
        D1[nc:, nc:] = self.G1
        D2 = np.zeros((m,) * 4)
        I = np.eye(nc)
        D2[:nc, :nc, :nc, :nc] = 4 * np.einsum("ik,jl->ijkl", I, I) - 2 * np.einsum("il,jk->ijkl", I, I)
        ca = slice(0, nc)
        ac = slice(nc, m)
        D2[ca, ac, ca, ac] = 2 * np.einsum("ij,tu->itju", I, self.G1)
        D2[ac, ca, ac, ca] = 2 * np.einsum("ij,tu->tiuj", I, self.G1)
        D2[ca, ac, ac, ca] = -np.einsum("ij,tu->ituj", I, self.G1)
        D2[ac, ca, ca, ac] = -np.einsum("ij,tu->tiju", I, self.G1)
        D2[ac, ac, ac, ac] = self.G2
        h = self.core_hamiltonian()[:m, :m]
        Bm = self.B[:, :m, :m]
        eri = np.einsum("Xpq,Xrs->pqrs", Bm, Bm)
        return float(np.einsum("pq,pq->", h, D1) + 0.5 * np.einsum("pqrs,prqs->", eri, D2))

    # --- residual and energy ------------------------------------------------------------
    def evaluator(self, T1, T2):
        sp = self.sp
        t1, t2 = spinorbital_amplitudes(sp, T1, T2)
        Hl = _hole_so(sp)
        Pl = _particle_so(sp)
        tens = dict(self.base)
        tens["t1"] = (t1, (list(range(2 * sp.n)),) * 2)
        tens["t2"] = (t2, (Hl, Hl, Pl, Pl))
        return Evaluator(sp, tens)

    def energy(self, T1, T2, variant="R1", groups=("lin", "quad")):
        """Correlation energy E_CC - E0 (filtered two-fold commutator)."""
        terms = term_lists(variant)
        ev = self.evaluator(T1, T2)
        e = 0.0
        if "lin" in groups:
            for t in terms["lin"]:
                if t.rank == 0:
                    e += float(ev.term(t, [], []))
        if "quad" in groups:
            for t in terms["quad_E"]:
                e += 0.5 * float(ev.term(t, [], []))
        return e

    def residual(self, T1, T2, variant="R1", groups=("lin", "quad")):
        """Spin-free residuals R1[H,P] (alpha) and R2[H,H,P,P] (alpha-beta sector)."""
        sp = self.sp
        terms = term_lists(variant)
        ev = self.evaluator(T1, T2)
        Hl, Pl = _hole_so(sp), _particle_so(sp)
        g1 = np.zeros((len(Pl), len(Hl)))
        g2 = np.zeros((len(Pl), len(Pl), len(Hl), len(Hl)))
        todo = []
        if "lin" in groups:
            todo += [(t, 1.0) for t in terms["lin"] if t.rank in (1, 2)]
        if "quad" in groups:
            todo += [(t, 0.5) for t in terms["quad_R"]]
        for t, scale in todo:
            U, L = t.upper(), t.lower()
            outs = [t.space[l] & P for l in U] + [t.space[l] & H for l in L]
            if not all(outs):
                continue
            val = ev.term(t, U + L, outs)
            if t.rank == 1:
                _scatter(sp, g1, (Pl, Hl), scale * val, outs)
            else:
                _scatter(sp, g2, (Pl, Pl, Hl, Hl), scale * val, outs)
        # eq. (antisym): Hbar^{pq}_{rs} = g^{pq}_{rs} - g^{qp}_{rs} - g^{pq}_{sr} + g^{qp}_{sr}
        h2 = g2 - g2.transpose(1, 0, 2, 3) - g2.transpose(0, 1, 3, 2) + g2.transpose(1, 0, 3, 2)
        nH, nP = sp.nH, sp.nP
        R1 = g1[:nP, :nH].T.copy()                              # alpha-alpha: r^c_k
        R2 = np.einsum("cdkl->klcd", h2[:nP, nP:, :nH, nH:])   # r^{c dbar}_{k lbar}
        na = sp.na
        R1[sp.nc:, :na] = 0.0                                  # TU left out
        R2[sp.nc:, sp.nc:, :na, :na] = 0.0                     # TUVW left out
        return R1, R2


def _hole_so(sp):
    return sp.so[C][:sp.nc] + sp.so[A][:sp.na] + sp.so[C][sp.nc:] + sp.so[A][sp.na:]


def _particle_so(sp):
    return sp.so[A][:sp.na] + sp.so[V][:sp.nv] + sp.so[A][sp.na:] + sp.so[V][sp.nv:]


# ----------------------------------------------------------------------------------------
# regularized Jacobi iteration


def denominators(f, nc, na, nv):
    """Delta for T1[k,c] and T2[k,l,c,d]: sum of hole minus particle diagonal Fock elements."""
    e = np.diag(f)
    eH = e[:nc + na]
    eP = e[nc:]
    D1 = eH[:, None] - eP[None, :]
    D2 = eH[:, None, None, None] + eH[None, :, None, None] - eP[None, None, :, None] - eP[None, None, None, :]
    return D1, D2


def regularizer(D, s):
    """(1 - exp(-s D^2)) / D, with its limit 0 at D = 0 (eq. ric-update)."""
    D = np.asarray(D, dtype=np.float64)
    out = np.zeros_like(D)
    nz = D != 0
    out[nz] = -np.expm1(-s * D[nz] ** 2) / D[nz]
    return out


def ric_update(T, R, D, s):
    """t <- (t Delta + r) (1 - exp(-s Delta^2)) / Delta (eq. ric-update)."""
    return (T * D + R) * regularizer(D, s)


def block_mask(nc, na, nv):
    """Masks of the amplitudes that exist (all-active blocks left out, Section 2.2)."""
    nH, nP = nc + na, na + nv
    m1 = np.ones((nH, nP), dtype=bool)
    m1[nc:, :na] = False
    m2 = np.ones((nH, nH, nP, nP), dtype=bool)
    m2[nc:, nc:, :na, :na] = False
    return m1, m2


def solve(ref: Reference, s: float, tol=1e-8, max_iter=200, variant="R1", T1=None, T2=None,
          callback=None):
    """Regularized Jacobi iteration from T = 0 until ||t_new - t|| < tol; returns (E_corr, T1, T2, it)."""
    sp = ref.sp
    D1, D2 = denominators(ref.f, sp.nc, sp.na, sp.nv)
    m1, m2 = block_mask(sp.nc, sp.na, sp.nv)
    if T1 is None:
        T1 = np.zeros((sp.nH, sp.nP))
        T2 = np.zeros((sp.nH, sp.nH, sp.nP, sp.nP))
    for it in range(1, max_iter + 1):
        R1, R2 = ref.residual(T1, T2, variant)
        N1 = ric_update(T1, R1, D1, s) * m1
        N2 = ric_update(T2, R2, D2, s) * m2
        step = math.sqrt(float(np.sum((N1 - T1) ** 2) + np.sum((N2 - T2) ** 2)))
        T1, T2 = N1, N2
        if callback is not None:
            callback(it, step, T1, T2)
        if step < tol:
            return ref.energy(T1, T2, variant), T1, T2, it
    raise RuntimeError("regularized iteration did not converge")
