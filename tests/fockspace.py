"""Brute-force Fock-space second quantization for tiny systems (test helper).

Independent of the oracle's Wick engine: operators act on explicit state
vectors over all 2^nso occupation-number states.  Spin-orbital index sigma*n + p.
Conventions follow Section 2.1 of the paper: a^{p1..pk}_{q1..qk} =
a^+_p1 .. a^+_pk a_qk .. a_q1, and generalized normal-ordered strings {..}
are defined by expanding an ordinary string into normal-ordered strings whose
coefficients are the reference RDMs of the removed operators.
"""
from __future__ import annotations

import itertools

import numpy as np


def _parity(order):
    inv = sum(1 for i in range(len(order)) for j in range(i + 1, len(order)) if order[j] < order[i])
    return -1 if inv % 2 else 1


class Fock:
    def __init__(self, nso: int):
        self.nso = nso
        self.dim = 1 << nso
        self.states = np.arange(self.dim, dtype=np.int64)

    # elementary operators on vectors ------------------------------------------------
    def ann(self, p: int, vec: np.ndarray) -> np.ndarray:
        s = self.states
        occ = (s >> p) & 1
        below = s & ((1 << p) - 1)
        sign = 1.0 - 2.0 * (self._popc(below) & 1)
        out = np.zeros_like(vec)
        src = s[occ == 1]
        out[src ^ (1 << p)] = vec[src] * sign[occ == 1]
        return out

    def cre(self, p: int, vec: np.ndarray) -> np.ndarray:
        s = self.states
        occ = (s >> p) & 1
        below = s & ((1 << p) - 1)
        sign = 1.0 - 2.0 * (self._popc(below) & 1)
        out = np.zeros_like(vec)
        src = s[occ == 0]
        out[src | (1 << p)] = vec[src] * sign[occ == 0]
        return out

    _pc = None

    def _popc(self, x):
        if Fock._pc is None or Fock._pc.size < self.dim:
            Fock._pc = np.array([bin(i).count("1") for i in range(max(self.dim, 1))], dtype=np.int64)
        return Fock._pc[x]

    def string(self, upper, lower, vec):
        """a^{upper}_{lower} |vec> = a^+_u1 .. a^+_uk a_lk .. a_l1 |vec>."""
        out = vec
        for q in lower:                  # a_l1 acts first
            out = self.ann(q, out)
        for p in reversed(upper):        # then a^+_uk ... a^+_u1
            out = self.cre(p, out)
        return out

    def basis_vector(self, occupied):
        """|occupied> = a^+_{o1} a^+_{o2} ... |vac> with o1 < o2 < ... ."""
        v = np.zeros(self.dim)
        v[0] = 1.0
        for p in sorted(occupied, reverse=True):
            v = self.cre(p, v)
        return v


class GNO:
    """Generalized normal-ordered strings with respect to a reference vector psi0."""

    def __init__(self, fock: Fock, psi0: np.ndarray, maxrank: int = 3):
        self.F = fock
        self.psi0 = psi0
        self._rdm = {}
        self._vec_cache = {}

    def rdm(self, upper, lower):
        key = (tuple(upper), tuple(lower))
        if key not in self._rdm:
            self._rdm[key] = float(self.psi0 @ self.F.string(upper, lower, self.psi0))
        return self._rdm[key]

    def apply(self, upper, lower, vec, vec_id):
        """{a^{upper}_{lower}} |vec>, recursively: ordinary string minus RDM-weighted lower strings."""
        key = (tuple(upper), tuple(lower), vec_id)
        if key in self._vec_cache:
            return self._vec_cache[key]
        k = len(upper)
        out = self.F.string(upper, lower, vec).copy()
        seq = [("c", u) for u in upper] + [("a", l) for l in reversed(lower)]
        cpos = list(range(k))
        apos = list(range(k, 2 * k))
        for m in range(1, k + 1):
            for I in itertools.combinations(cpos, m):
                for J in itertools.combinations(apos, m):
                    rest_c = [i for i in cpos if i not in I]
                    rest_a = [j for j in apos if j not in J]
                    order = list(I) + list(J) + rest_c + rest_a
                    sign = _parity(order)
                    g_up = [seq[i][1] for i in I]
                    g_lo = [seq[j][1] for j in J][::-1]
                    g = self.rdm(g_up, g_lo)
                    if g == 0.0:
                        continue
                    r_up = [seq[i][1] for i in rest_c]
                    r_lo = [seq[j][1] for j in rest_a][::-1]
                    if r_up:
                        out = out - sign * g * self.apply(r_up, r_lo, vec, vec_id)
                    else:
                        out = out - sign * g * vec
        self._vec_cache[key] = out
        return out

    def operator_apply(self, coeffs: dict, vec, vec_id):
        """sum over ranks r of sum_{U,L} coeffs[r][U,L] {a^U_L} |vec>, every index tuple summed.

        coeffs[r] is an array over (nso,)*(2r); rank 0 is a scalar.  The strings of one set
        of indices differ only by the sign of the reordering, so the sum is taken over
        increasing tuples U, L with the signed sum of the coefficients of their orderings.
        """
        out = np.zeros_like(vec)
        nso = self.F.nso
        for r, G in coeffs.items():
            if r == 0:
                out = out + float(G) * vec
                continue
            combs, Gc = combination_coefficients(G, r, nso)
            for iu, il in zip(*np.nonzero(Gc)):
                out = out + Gc[iu, il] * self.apply(list(combs[iu]), list(combs[il]), vec, vec_id)
        return out


def combination_coefficients(G, r, nso):
    """Increasing r-tuples of range(nso) and, for each pair (U, L) of them, the signed sum of
    G over every reordering of U and of L: the value antisymmetrize(G) takes at (U, L)."""
    combs = list(itertools.combinations(range(nso), r))
    idx = np.array(combs, dtype=np.int64).reshape(len(combs), r)
    perms = list(itertools.permutations(range(r)))
    out = np.zeros((len(combs), len(combs)))
    for pu in perms:
        su = _parity(list(pu))
        U = idx[:, list(pu)]
        for pl in perms:
            sl = _parity(list(pl))
            L = idx[:, list(pl)]
            sel = tuple(U[:, None, i] for i in range(r)) + tuple(L[None, :, i] for i in range(r))
            out += su * sl * G[sel]
    return combs, out


def antisymmetrize(G):
    """sum over permutations of upper and of lower indices with parity (no 1/k! factors)."""
    r = G.ndim // 2
    out = np.zeros_like(G)
    for pu in itertools.permutations(range(r)):
        for pl in itertools.permutations(range(r)):
            sg = _parity(list(pu)) * _parity(list(pl))
            out += sg * np.transpose(G, list(pu) + [r + i for i in pl])
    return out


def spin_orbital_integrals(B, n):
    """v^{pq}_{rs} = <pq||rs> over spin orbitals sigma*n + p from B[X,p,q]."""
    eri = np.einsum("Xpq,Xrs->pqrs", B, B)          # (pq|rs)
    so = np.zeros((2 * n,) * 4)
    for s1 in (0, 1):
        for s2 in (0, 1):
            a, b = slice(s1 * n, s1 * n + n), slice(s2 * n, s2 * n + n)
            # <pq|rs> = (pr|qs) delta(s_p,s_r) delta(s_q,s_s)
            so[a, b, a, b] += np.einsum("prqs->pqrs", eri)
            so[a, b, b, a] -= np.einsum("psqr->pqrs", eri)
    return so


class Hamiltonian:
    """H = sum h^p_q a^p_q + 1/4 sum v^{pq}_{rs} a^{pq}_{rs} applied to vectors (ordinary strings)."""

    def __init__(self, fock: Fock, h_so: np.ndarray, v_so: np.ndarray):
        self.F = fock
        self.h = h_so
        self.v = v_so

    def _epq(self, p, q, vec):
        return self.F.cre(p, self.F.ann(q, vec))

    def apply(self, vec):
        # a^+_p a^+_q a_s a_r = E_pr E_qs - delta_qr E_ps with E_pq = a^+_p a_q
        nso = self.F.nso
        W = np.array([[self._epq(q, s, vec) for s in range(nso)] for q in range(nso)])
        acc = self.h[:, :, None] * vec[None, None, :] + 0.25 * np.einsum("pqrs,qsd->prd", self.v, W)
        out = np.zeros_like(vec)
        for p in range(nso):
            for r in range(nso):
                out += self._epq(p, r, acc[p, r])
        x = -0.25 * np.einsum("pqqs->ps", self.v)
        out += np.einsum("ps,psd->d", x, W)
        return out


def embed_reference(fock: Fock, nc: int, na: int, n: int, dets, coeffs):
    """Psi0 = core (doubly occupied) x CAS vector; active spatial t -> spin orbital sigma*n + nc + t."""
    psi = np.zeros(fock.dim)
    core = [s * n + i for s in (0, 1) for i in range(nc)]
    for d, c in zip(dets, coeffs):
        occ = list(core)
        for s in (0, 1):
            for t in range(na):
                if (int(d) >> (t + s * na)) & 1:
                    occ.append(s * n + nc + t)
        psi += c * fock.basis_vector(occ)
    return psi / np.linalg.norm(psi)
