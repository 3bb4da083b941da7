"""Reference interpreter of the library's contraction plan with numpy (test helper only).

It executes the same plan text the HIP runtime executes, so that the plan
produced by the library's equation generator can be checked against the
oracle on the CPU before any GPU run.  It is not part of the product path.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _offsets(nc, na, nv, naux):
    n = nc + na + nv
    nH, nP = nc + na, na + nv
    sub = {
        "G": {"C": (0, nc), "A": (nc, nc + na), "V": (nc + na, n), "H": (0, nH), "P": (nc, n), "G": (0, n)},
        "H": {"C": (0, nc), "A": (nc, nH), "H": (0, nH)},
        "P": {"A": (0, na), "V": (na, nP), "P": (0, nP)},
        "A": {"A": (0, na)},
        "C": {"C": (0, nc)},
        "V": {"V": (0, nv)},
        "X": {"X": (0, naux)},
    }
    ext = {"C": nc, "A": na, "V": nv, "H": nH, "P": nP, "G": n, "X": naux}
    return sub, ext


DECL = {
    "f": "GG", "B": "XGG", "T1": "HP", "T2": "HHPP", "gA": "AA", "eA": "AA", "K2": "AAAA",
    "K3": "AAAAAA", "I4": "HHHH", "I3": "HHHP", "IJ": "HHPP", "IK": "HPHP",
    "R1": "HP", "R2": "HHPP", "TAU": "HHPP", "E": "",
    "XR1": "HP", "XL": "HHPP", "YL": "HHPP", "dT1": "HP", "dT2": "HHPP", "dF": "GG", "dB": "XGG",
    "dI4": "HHHH", "dI3": "HHHP", "dIJ": "HHPP", "dIK": "HPHP",
}


def prepare(f, B, G1, G2, G3, nc, na, nv):
    """Tensors the runtime prepares once per problem (written from the same definitions)."""
    n = nc + na + nv
    nH = nc + na
    e = np.einsum
    out = {"f": f, "B": B}
    if na:
        g = 0.5 * G1
        out["gA"] = g
        out["eA"] = np.eye(na) - g
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
        out["K2"] = (2 * L2 + e("pqsr->pqrs", L2)) / 6.0
        K3 = (17 * L3
              - e("pqrtsu->pqrstu", L3) - e("pqruts->pqrstu", L3) - e("pqrsut->pqrstu", L3)
              - 7 * e("pqrtus->pqrstu", L3) - 7 * e("pqrust->pqrstu", L3)) / 144.0
        out["K3"] = K3
    else:
        out["gA"] = out["eA"] = np.zeros((0, 0))
        out["K2"] = np.zeros((0,) * 4)
        out["K3"] = np.zeros((0,) * 6)
    BH = B[:, :nH, :nH]
    BHP = B[:, :nH, nc:]
    BPP = B[:, nc:, nc:]
    out["I4"] = e("xpr,xqs->prqs", BH, BH)
    out["I3"] = e("xpr,xqs->prqs", BH, BHP)
    out["IJ"] = e("xpr,xqs->prqs", BH, BPP)
    out["IK"] = e("xpr,xqs->prqs", BHP, BHP)
    return out


class Interpreter:
    def __init__(self, plan_text, nc, na, nv, naux):
        self.lines = [l.strip() for l in plan_text.splitlines() if l.strip() and not l.startswith("#")]
        self.sub, self.ext = _offsets(nc, na, nv, naux)
        self.nc, self.na, self.nv = nc, na, nv
        self.decl = dict(DECL)

    def view(self, T, operand):
        name, rngs, labs = operand.split(":")
        arr = T[name]
        decl = self.decl[name]
        idx = []
        for d, r in zip(decl, rngs):
            a, b = self.sub[d][r]
            idx.append(slice(a, b))
        return arr[tuple(idx)] if idx else arr, labs.split(",") if labs else []

    def run(self, section, tensors):
        T = tensors
        active = False
        for line in self.lines:
            tok = line.split()
            if tok[0] == "SECTION":
                active = tok[1] == section
                continue
            if not active:
                continue
            op = tok[0]
            if op == "END":
                break
            if op == "ALLOC":
                self.decl[tok[1]] = tok[2]
                T[tok[1]] = np.zeros(tuple(self.ext[c] for c in tok[2]))
            elif op == "FREE":
                T.pop(tok[1], None)
            elif op == "ZERO":
                if tok[1] == "E":
                    T["E"] = np.zeros(())
                else:
                    T[tok[1]][...] = 0.0
            elif op in ("CONTRACT", "CONTRACT0"):
                alpha = float(Fraction(tok[1]))
                ov, ol = self.view(T, tok[2])
                av, al = self.view(T, tok[3])
                bv, bl = self.view(T, tok[4])
                letters = {}
                for l in ol + al + bl:
                    if l not in letters:
                        letters[l] = chr(ord("a") + len(letters)) if len(letters) < 26 else chr(ord("A") + len(letters) - 26)
                spec = "".join(letters[l] for l in al) + "," + "".join(letters[l] for l in bl) + "->" + "".join(letters[l] for l in ol)
                ov += alpha * np.einsum(spec, av, bv, optimize=True)
            elif op == "ADD":
                alpha = float(Fraction(tok[1]))
                ov, ol = self.view(T, tok[2])
                av, al = self.view(T, tok[3])
                letters = {l: chr(ord("a") + i) for i, l in enumerate(dict.fromkeys(ol + al))}
                spec = "".join(letters[l] for l in al) + "->" + "".join(letters[l] for l in ol)
                ov += alpha * np.einsum(spec, av)
            elif op == "DFC":
                alpha = float(Fraction(tok[1]))
                ov, ol = self.view(T, tok[2])
                l1, ll1 = self.view(T, tok[3])
                l2, ll2 = self.view(T, tok[4])
                yv, yl = self.view(T, tok[5])
                eri = np.einsum("xpr,xqs->prqs", l1, l2)
                el = ll1[1:] + ll2[1:]
                letters = {l: chr(ord("a") + i) for i, l in enumerate(dict.fromkeys(ol + el + yl))}
                spec = ("".join(letters[l] for l in el) + "," + "".join(letters[l] for l in yl) + "->"
                        + "".join(letters[l] for l in ol))
                ov += alpha * np.einsum(spec, eri, yv, optimize=True)
            elif op == "SYMMETRIZE":
                x = T[tok[1]]
                x[...] = x + x.transpose(1, 0, 3, 2)
            elif op == "SYMHALF":
                x = T[tok[1]]
                x[...] = 0.5 * (x + x.transpose(1, 0, 3, 2))
            elif op == "LADDER":
                nc = self.nc
                Bp = T["B"][:, nc:, nc:]
                W = np.einsum("xce,xdf->cedf", Bp, Bp)
                T[tok[1]] += np.einsum("cedf,klef->klcd", W, T[tok[2]], optimize=True)
            elif op == "LADDERGRAD":
                # dB[X,c,e] += 2 sum_{d,f} V[c,e,d,f] B[X,d,f],  V = sum_kl XL[k,l,c,d] tau[k,l,e,f]
                nc = self.nc
                Bp = T["B"][:, nc:, nc:]
                V = np.einsum("klcd,klef->cedf", T[tok[2]], T[tok[3]], optimize=True)
                T[tok[1]][:, nc:, nc:] += 2.0 * np.einsum("cedf,xdf->xce", V, Bp, optimize=True)
            elif op in ("LOOP", "ENDLOOP"):
                pass   # chunking does not change what is computed
            elif op == "MASK":
                nc, na = self.nc, self.na
                T[tok[1]][nc:, :na] = 0.0
                T[tok[2]][nc:, nc:, :na, :na] = 0.0
            else:
                raise ValueError(op)
        return T
