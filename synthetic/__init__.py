"""Seeded synthetic inputs for the spin-free RIC-MRCCSD residual.

This module is shared by the CPU oracle, the tests, the benchmark and the
smoke check.  It holds no arithmetic of the method itself: it only draws the
inputs the method consumes (Section 2.1 and 2.2 of the paper):

* orbital energies and a generalized Fock matrix f (core, active, virtual
  ordering; Table 1 of the paper for the spaces),
* density-fitting factors B[P,p,q] with (pq|rs) = sum_P B[P,p,q] B[P,r,s],
* a CAS vector over all M_S = 0 determinants of CAS(na, na) and its
  spin-free 1-, 2- and 3-body reduced density matrices
  Gamma^{PQ..}_{RS..} = sum over spins <a^+_{P s1} a^+_{Q s2} .. a_{S s2} a_{R s1}>
  (the spin-integrated RDMs of Section 2.3.2).

Recipe (all configurations): numpy.random.default_rng(seed); draw order is
orbital energies -> Fock off-diagonal -> B -> CI vector.
  eps ~ U[-20,-0.5] (core), U[-0.5,0.5] (active), U[0.5,5] (virtual)
  f = diag(eps) + symmetric off-diagonal noise with standard deviation 1e-2
  B[P,p,q] = z/((1+|p-q|) sqrt(naux)), z ~ N(0,1), symmetric in (p,q) by
             mirroring the upper triangle (diagonal included)
  CI vector: N(0,1) on every M_S=0 determinant (dense) or on a uniformly
             chosen fraction of them (sparse), then normalized.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from math import comb

import numpy as np

__all__ = [
    "Config", "CONFIGS", "Inputs", "make_inputs", "make_fock", "make_df",
    "cas_determinants", "random_ci", "spinfree_rdms", "spinorbital_rdms",
    "project_singlet", "popcount",
]


@dataclass(frozen=True)
class Config:
    name: str
    nc: int
    na: int
    nv: int
    naux: int
    seed: int
    ci_fraction: float = 1.0     # 1.0 = dense CI vector
    s: float = 0.5               # flow parameter (E_h^-2)
    tol: float = 1e-8
    max_iter: int = 200

    @property
    def n(self) -> int:
        return self.nc + self.na + self.nv


# Workloads: sizes of the paper's systems scaled as stated by each name.
CONFIGS = {
    "tiny_cas44": Config("tiny_cas44", nc=2, na=4, nv=10, naux=48, seed=1),
    "mixed_cas88": Config("mixed_cas88", nc=10, na=8, nv=120, naux=360, seed=2),
    "adjoint_cas66": Config("adjoint_cas66", nc=6, na=6, nv=60, naux=180, seed=3),
    "large_cas1414": Config("large_cas1414", nc=20, na=14, nv=300, naux=900, seed=4,
                            ci_fraction=0.01),
    "b12_cas1212": Config("b12_cas1212", nc=40, na=12, nv=757, naux=2200, seed=5,
                          ci_fraction=0.01),
}


@dataclass
class Inputs:
    cfg: Config
    f: np.ndarray            # (n, n) generalized Fock matrix, symmetric
    B: np.ndarray            # (naux, n, n) DF factors, symmetric in (p, q)
    G1: np.ndarray           # (na, na) spin-free 1-RDM (active block)
    G2: np.ndarray           # (na,)*4  Gamma^{PQ}_{RS} stored as G2[P,Q,R,S]
    G3: np.ndarray           # (na,)*6  Gamma^{PQR}_{STU} stored as G3[P,Q,R,S,T,U]
    dets: np.ndarray = field(repr=False, default=None)
    coeffs: np.ndarray = field(repr=False, default=None)


def popcount(x: np.ndarray) -> np.ndarray:
    """Bit count of each element of an unsigned 64-bit array."""
    x = np.asarray(x, dtype=np.uint64)
    c = np.zeros(x.shape, dtype=np.int64)
    y = x.copy()
    while np.any(y):
        c += (y & np.uint64(1)).astype(np.int64)
        y >>= np.uint64(1)
    return c


def make_fock(rng: np.random.Generator, nc: int, na: int, nv: int) -> np.ndarray:
    eps = np.concatenate([
        rng.uniform(-20.0, -0.5, nc),
        rng.uniform(-0.5, 0.5, na),
        rng.uniform(0.5, 5.0, nv),
    ])
    n = nc + na + nv
    z = rng.normal(0.0, 1e-2, (n, n))
    off = np.triu(z, 1)
    return np.diag(eps) + off + off.T


def make_df(rng: np.random.Generator, n: int, naux: int) -> np.ndarray:
    """B[P,p,q] = z/((1+|p-q|) sqrt(naux)), z symmetric N(0,1); built slice by slice."""
    idx = np.arange(n)
    scale = 1.0 / ((1.0 + np.abs(idx[:, None] - idx[None, :])) * np.sqrt(naux))
    B = np.empty((naux, n, n))
    for P in range(naux):
        z = rng.standard_normal((n, n))
        u = np.triu(z)
        B[P] = (u + np.triu(z, 1).T) * scale
    return B


def cas_determinants(na: int, nalpha: int | None = None, nbeta: int | None = None) -> np.ndarray:
    """All determinants of CAS(N, na) with the given alpha/beta counts (default M_S = 0, N = na).

    A determinant is a 2*na bit string: bits 0..na-1 are alpha spin-orbitals,
    bits na..2na-1 are beta spin-orbitals (spin-orbital index p + sigma*na).
    """
    if nalpha is None:
        nalpha = na // 2
    if nbeta is None:
        nbeta = na - nalpha
    astr = [sum(1 << i for i in c) for c in itertools.combinations(range(na), nalpha)]
    bstr = [sum(1 << i for i in c) for c in itertools.combinations(range(na), nbeta)]
    dets = np.array([a | (b << na) for a in astr for b in bstr], dtype=np.uint64)
    return dets


def random_ci(rng: np.random.Generator, na: int, fraction: float = 1.0):
    """Random normalized M_S = 0 CI vector; returns (dets, coeffs) of the non-zeros."""
    dets = cas_determinants(na)
    ndet = dets.size
    if fraction >= 1.0:
        c = rng.standard_normal(ndet)
        keep = dets
    else:
        nnz = max(1, int(round(fraction * ndet)))
        pos = np.sort(rng.choice(ndet, size=nnz, replace=False))
        keep = dets[pos]
        c = rng.standard_normal(nnz)
    c = c / np.linalg.norm(c)
    return keep, c


def _annihilate(dets, amps, codes, q: int, nbits: int):
    """Apply a_q to every entry (det, amp, tuple code); drop entries where q is empty."""
    bit = np.uint64(1) << np.uint64(q)
    occ = (dets & bit) != 0
    d = dets[occ]
    a = amps[occ]
    below = d & (bit - np.uint64(1))
    sign = np.where(popcount(below) % 2 == 0, 1.0, -1.0)
    return d ^ bit, a * sign, codes[occ]


def _annihilation_table(dets, coeffs, nso: int, k: int):
    """Entries of phi_(q1..qk) = a_qk .. a_q1 |Psi> as (det, amp, tuple code).

    The tuple code is q1*nso^(k-1) + ... + qk.
    """
    cur = [(dets.astype(np.uint64), coeffs.astype(np.float64), np.zeros(dets.size, dtype=np.int64))]
    for _ in range(k):
        nxt = []
        for d, a, c in cur:
            for q in range(nso):
                d2, a2, c2 = _annihilate(d, a, c, q, nso)
                if d2.size:
                    nxt.append((d2, a2, c2 * nso + q))
        cur = nxt
    if not cur:
        return (np.zeros(0, dtype=np.uint64), np.zeros(0), np.zeros(0, dtype=np.int64))
    d = np.concatenate([x[0] for x in cur])
    a = np.concatenate([x[1] for x in cur])
    c = np.concatenate([x[2] for x in cur])
    return d, a, c


def _gram(d, a, c, ncol: int) -> np.ndarray:
    """Dense M^T M where M[det, code] = amp (entries with equal (det, code) summed)."""
    import scipy.sparse as sp
    if d.size == 0:
        return np.zeros((ncol, ncol))
    _, row = np.unique(d, return_inverse=True)
    M = sp.csr_matrix((a, (row, c)), shape=(row.max() + 1, ncol))
    return (M.T @ M).toarray()


def spinorbital_rdms(dets, coeffs, na: int, kmax: int = 3):
    """Spin-orbital RDMs gamma^{p1..pk}_{q1..qk} = <a^+_p1..a^+_pk a_qk..a_q1>, k = 1..kmax.

    Spin-orbital index p + sigma*na; returns a list of arrays of shape (2na,)*(2k).
    """
    nso = 2 * na
    out = []
    for k in range(1, kmax + 1):
        d, a, c = _annihilation_table(dets, coeffs, nso, k)
        g = _gram(d, a, c, nso ** k)
        out.append(g.reshape((nso,) * (2 * k)))
    return out


def _annihilation_table_sorted(dets, coeffs, nso: int, k: int):
    """Entries of a_qk .. a_q1 |Psi> for increasing q1 < .. < qk only, as (det, amp, tuple code)."""
    cur = [(dets.astype(np.uint64), coeffs.astype(np.float64), np.zeros(dets.size, dtype=np.int64), -1)]
    for _ in range(k):
        nxt = []
        for d, a, c, last in cur:
            for q in range(last + 1, nso):
                d2, a2, c2 = _annihilate(d, a, c, q, nso)
                if d2.size:
                    nxt.append((d2, a2, c2 * nso + q, q))
        cur = nxt
    if not cur:
        return (np.zeros(0, dtype=np.uint64), np.zeros(0), np.zeros(0, dtype=np.int64))
    return (np.concatenate([x[0] for x in cur]), np.concatenate([x[1] for x in cur]),
            np.concatenate([x[2] for x in cur]))


def spinfree_rdms(dets, coeffs, na: int, kmax: int = 3):
    """Spin-free RDMs Gamma^{P1..Pk}_{Q1..Qk} summed over column spins, k = 1..kmax.

    The spin-orbital RDM is formed over increasing index tuples only (the Gram matrix of
    a_qk .. a_q1 |Psi> for q1 < .. < qk); an element with its indices in another order is that
    value times the sign of the sorting permutation, and repeated indices give zero.
    """
    nso = 2 * na
    out = []
    for k in range(1, kmax + 1):
        d, a, c = _annihilation_table_sorted(dets, coeffs, nso, k)
        codes, col = np.unique(c, return_inverse=True) if c.size else (np.zeros(0, dtype=np.int64), c)
        g = _gram(d, a, col, max(codes.size, 1))
        # column of every ordered spin-orbital tuple: (spatial tuple, spin pattern) -> (sorted column, sign)
        where = {int(x): i for i, x in enumerate(codes)}
        nsp = na ** k
        G = np.zeros((nsp, nsp))
        for pat in itertools.product((0, 1), repeat=k):
            cols = np.full(nsp, -1, dtype=np.int64)
            sgn = np.zeros(nsp)
            for j, P in enumerate(itertools.product(range(na), repeat=k)):
                q = [P[i] + pat[i] * na for i in range(k)]
                if len(set(q)) < k:
                    continue
                order = sorted(range(k), key=lambda i: q[i])
                inv = sum(1 for x in range(k) for y in range(x + 1, k) if order[y] < order[x])
                code = 0
                for i in order:
                    code = code * nso + q[i]
                if code in where:
                    cols[j] = where[code]
                    sgn[j] = -1.0 if inv % 2 else 1.0
            ok = cols >= 0
            if not np.any(ok):
                continue
            sub = g[np.ix_(cols[ok], cols[ok])] * np.outer(sgn[ok], sgn[ok])
            G[np.ix_(ok, ok)] += sub
        out.append(G.reshape((na,) * (2 * k)))
    return out


def spinfree_rdms_ordered(dets, coeffs, na: int, kmax: int = 3):
    """Spin-free RDMs Gamma^{P1..Pk}_{Q1..Qk} summed over column spins, k = 1..kmax.

    Gamma[P1..Pk, Q1..Qk] = sum_{s1..sk} <a^+_{P1 s1} .. a^+_{Pk sk} a_{Qk sk} .. a_{Q1 s1}>.
    """
    nso = 2 * na
    out = []
    for k in range(1, kmax + 1):
        d, a, c = _annihilation_table(dets, coeffs, nso, k)
        # decode spin pattern and spatial code of every tuple
        digits = []
        cc = c.copy()
        for _ in range(k):
            digits.append(cc % nso)
            cc //= nso
        digits = digits[::-1]                      # q1 .. qk
        spins = np.zeros(c.size, dtype=np.int64)
        spat = np.zeros(c.size, dtype=np.int64)
        for q in digits:
            spins = spins * 2 + (q // na)
            spat = spat * na + (q % na)
        G = np.zeros((na ** k, na ** k))
        for sp_pat in range(2 ** k):
            m = spins == sp_pat
            if np.any(m):
                G += _gram(d[m], a[m], spat[m], na ** k)
        out.append(G.reshape((na,) * (2 * k)))
    return out


def _s2_matrix(dets: np.ndarray, na: int) -> np.ndarray:
    """S^2 in the determinant basis (same N, M_S), by explicit second quantization."""
    index = {int(d): i for i, d in enumerate(dets)}
    n = dets.size
    S2 = np.zeros((n, n))
    for i, d in enumerate(dets):
        d = int(d)
        na_ = bin(d & ((1 << na) - 1)).count("1")
        nb_ = bin(d >> na).count("1")
        ms = 0.5 * (na_ - nb_)
        # S^2 = S- S+ + Sz^2 + Sz ; S+ = sum_p a^+_{p a} a_{p b}
        S2[i, i] += ms * ms + ms
        # S- S+ |d> : apply S+ then S-
        for p in range(na):
            ob, oa = na + p, p
            if not (d >> ob) & 1 or (d >> oa) & 1:
                continue
            s1 = (-1) ** bin(d & ((1 << ob) - 1)).count("1")
            d1 = d ^ (1 << ob)
            s1 *= (-1) ** bin(d1 & ((1 << oa) - 1)).count("1")
            d1 |= (1 << oa)
            for q in range(na):
                qa, qb = q, na + q
                if not (d1 >> qa) & 1 or (d1 >> qb) & 1:
                    continue
                s2 = (-1) ** bin(d1 & ((1 << qa) - 1)).count("1")
                d2 = d1 ^ (1 << qa)
                s2 *= (-1) ** bin(d2 & ((1 << qb) - 1)).count("1")
                d2 |= (1 << qb)
                S2[index[d2], i] += s1 * s2
    return S2


def project_singlet(rng: np.random.Generator, na: int):
    """A random normalized S = 0 vector of CAS(na, na) (dense; small na only)."""
    dets = cas_determinants(na)
    S2 = _s2_matrix(dets, na)
    w, V = np.linalg.eigh(S2)
    null = V[:, np.abs(w) < 1e-8]
    c = null @ rng.standard_normal(null.shape[1])
    return dets, c / np.linalg.norm(c)


def spin_lower(dets, coeffs, na: int):
    """S_- |Psi> with S_- = sum_p a^+_{p beta} a_{p alpha}; returns (dets, coeffs)."""
    out = {}
    for d, c in zip(dets, coeffs):
        d = int(d)
        for p in range(na):
            oa, ob = p, na + p
            if not (d >> oa) & 1 or (d >> ob) & 1:
                continue
            s = (-1) ** bin(d & ((1 << oa) - 1)).count("1")
            d1 = d ^ (1 << oa)
            s *= (-1) ** bin(d1 & ((1 << ob) - 1)).count("1")
            d1 |= 1 << ob
            out[d1] = out.get(d1, 0.0) + s * float(c)
    keys = sorted(out)
    return np.array(keys, dtype=np.uint64), np.array([out[k] for k in keys])


def random_triplet(rng: np.random.Generator, na: int):
    """A random normalized S = 1, M_S = 1 vector of CAS(na, na) and its M_S = 0 partner
    S_-|Psi> / |S_-|Psi>| (dense; small na only).  Returns ((dets1, c1), (dets0, c0))."""
    dets = cas_determinants(na, na // 2 + 1, na - na // 2 - 1)
    S2 = _s2_matrix(dets, na)
    w, V = np.linalg.eigh(S2)
    sub = V[:, np.abs(w - 2.0) < 1e-8]
    c = sub @ rng.standard_normal(sub.shape[1])
    c = c / np.linalg.norm(c)
    d0, c0 = spin_lower(dets, c, na)
    return (dets, c), (d0, c0 / np.linalg.norm(c0))


def make_inputs(cfg: Config, with_rdms: bool = True) -> Inputs:
    rng = np.random.default_rng(cfg.seed)
    f = make_fock(rng, cfg.nc, cfg.na, cfg.nv)
    B = make_df(rng, cfg.n, cfg.naux)
    na = cfg.na
    if na == 0:
        z = np.zeros((0,) * 2)
        return Inputs(cfg, f, B, z, np.zeros((0,) * 4), np.zeros((0,) * 6))
    dets, c = random_ci(rng, na, cfg.ci_fraction)
    if with_rdms:
        G1, G2, G3 = spinfree_rdms(dets, c, na, 3)
    else:
        G1 = G2 = G3 = None
    return Inputs(cfg, f, B, G1, G2, G3, dets, c)


def custom_config(name: str, nc: int, na: int, nv: int, naux: int, seed: int, **kw) -> Config:
    return Config(name, nc=nc, na=na, nv=nv, naux=naux, seed=seed, **kw)


def ndets(na: int) -> int:
    return comb(na, na // 2) * comb(na, na - na // 2)
