"""Plan compiler: spin-free terms -> a list of tensor operations for the HIP runtime.

Build-time tool.  Input: the spin-free terms of E_corr, R1 and S2 from
algebra.derive().  Output: a text plan (one operation per line) that the C++
runtime parses at set-up and executes with the library's kernels.

Tensors and their axis ranges (C core, A active, V virtual, H = C+A, P = A+V,
G = all orbitals, X = auxiliary DF index):
  inputs   f(G,G)  B(X,G,G)  T1(H,P)  T2(H,H,P,P)
  prepared gA(A,A) = Gamma1/2, eA(A,A) = 1 - Gamma1/2, K2(A^4), K3(A^6),
           I4(H,H,H,H) I3(H,H,H,P) IJ(H,H,P,P) IK(H,P,H,P): (pr|qs) blocks with at
           most two particle indices, built once from B
  outputs  R1(H,P)  R2(H,H,P,P)  E (scalar)
Two-electron integrals with three or four particle indices are never formed:
they are contracted through B.  The terms of the particle-particle ladder
sum_{ef} (ce|df) Y[k,l,e,f] are collected into one tau(H,H,P,P) and applied by
the LADDER operation, which builds (ce|df) from B in chunks.

Every other term is factorized greedily into binary contractions; terms whose
last contraction pairs the same stored tensor with the same index pattern share
one accumulated intermediate ("sum before contract").
"""
from __future__ import annotations

import itertools
from collections import OrderedDict
from fractions import Fraction

from .algebra import A, C, G, H, P, V, RANGE_NAME, SFTerm

X = 8          # auxiliary range mask (not an orbital space)
RN = dict(RANGE_NAME)
RN[X] = "X"
SMALL = (C, A, H)
BIG = (V, P, G)

# representative sizes for the cost model (the 809-orbital CAS(12,12) shape)
COST_SIZES = {"nc": 40, "na": 12, "nv": 757, "naux": 2200}


def extent(r, sz=COST_SIZES):
    nc, na, nv, nx = sz["nc"], sz["na"], sz["nv"], sz["naux"]
    return {C: nc, A: na, V: nv, H: nc + na, P: na + nv, G: nc + na + nv, X: nx}[r]


# declared axis ranges of stored tensors
DECL = {
    "f": (G, G), "B": (X, G, G), "T1": (H, P), "T2": (H, H, P, P),
    "gA": (A, A), "eA": (A, A), "K2": (A,) * 4, "K3": (A,) * 6,
    "I4": (H, H, H, H), "I3": (H, H, H, P), "IJ": (H, H, P, P), "IK": (H, P, H, P),
    "R1": (H, P), "R2": (H, H, P, P), "TAU": (H, H, P, P),
    # adjoint sections: cotangents, the ladder applied to XL, and gradient outputs
    "XR1": (H, P), "XL": (H, H, P, P), "YL": (H, H, P, P),
    "dT1": (H, P), "dT2": (H, H, P, P), "dF": (G, G), "dB": (X, G, G),
    "dI4": (H, H, H, H), "dI3": (H, H, H, P), "dIJ": (H, H, P, P), "dIK": (H, P, H, P),
}


def parent(r):
    return H if r in SMALL else P


def _widen(r):
    """Core widens to the hole range, virtual to the particle range; others stay."""
    return {C: H, V: P}.get(r, r)


class Operand:
    __slots__ = ("name", "ranges", "labels", "src")

    def __init__(self, name, ranges, labels):
        self.name = name
        self.ranges = tuple(ranges)
        self.labels = tuple(labels)
        self.src = None

    def size(self):
        n = 1
        for r in self.ranges:
            n *= extent(r)
        return n

    def text(self):
        return f"{self.name}:{''.join(RN[r] for r in self.ranges)}:{','.join(str(l) for l in self.labels)}"


def _eri_operand(labels, rng):
    """(pr|qs) factor with labels (p,r,q,s) -> stored block operand, or None if it must use B."""
    p, r, q, s = labels
    par = [parent(rng[x]) for x in labels]
    nbig = sum(1 for x in par if x == P)
    if nbig > 2:
        return None
    # canonical blocks: I4 (HH|HH), I3 (HH|HP), IJ (HH|PP), IK (HP|HP)
    cands = []
    perms = [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
             (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)]
    table = {(H, H, H, H): "I4", (H, H, H, P): "I3", (H, H, P, P): "IJ", (H, P, H, P): "IK"}
    for pm in perms:
        pp = tuple(par[i] for i in pm)
        if pp in table:
            ls = tuple(labels[i] for i in pm)
            cands.append(Operand(table[pp], [rng[x] for x in ls], ls))
    return cands[0]


class Plan:
    def __init__(self):
        self.lines = []
        self.tmp = 0
        self.flops = 0.0
        self.ladder_flops = 0.0

    def new_tmp(self, ranges):
        name = f"t{self.tmp}"
        self.tmp += 1
        self.lines.append(f"ALLOC {name} {''.join(RN[r] for r in ranges)}")
        return name

    def free(self, name):
        self.lines.append(f"FREE {name}")

    def contract(self, out: Operand, alpha, a: Operand, b: Operand, fresh=False):
        labs = set(a.labels) | set(b.labels)
        rng = {}
        for o in (a, b, out):
            for l, r in zip(o.labels, o.ranges):
                rng[l] = r
        fl = 2.0
        for l in labs:
            fl *= extent(rng[l])
        self.flops += fl
        kind = "CONTRACT0" if fresh else "CONTRACT"
        self.lines.append(f"{kind} {_num(alpha)} {out.text()} {a.text()} {b.text()}")

    def add(self, out: Operand, alpha, a: Operand):
        self.lines.append(f"ADD {_num(alpha)} {out.text()} {a.text()}")


def _num(x):
    x = Fraction(x)
    return f"{x.numerator}/{x.denominator}"


def factor_operands(t: SFTerm):
    """Operands of a spin-free term after choosing integral blocks / DF factors."""
    ops = []
    aux = 0
    for name, ls in t.factors:
        if name == "eri":
            o = _eri_operand(ls, t.rng)
            if o is not None:
                ops.append(o)
            else:
                p, r, q, s = ls
                xl = f"X{aux}"
                aux += 1
                ops.append(Operand("B", (X, t.rng[p], t.rng[r]), (xl, p, r)))
                ops.append(Operand("B", (X, t.rng[q], t.rng[s]), (xl, q, s)))
        else:
            ops.append(Operand(name, [t.rng[l] for l in ls], ls))
    return ops


def _rng_of(ops, out_labels=(), out_ranges=()):
    r = {}
    for o in ops:
        for l, x in zip(o.labels, o.ranges):
            r[l] = x
    for l, x in zip(out_labels, out_ranges):
        r[l] = x
    return r


def _pair_cost(a, b, keep, rng):
    labs = set(a.labels) | set(b.labels)
    fl = 1.0
    for l in labs:
        fl *= extent(rng[l])
    for o in (a, b):
        if o.name == "ERI":           # the integral block is built from its DF factors
            fb = extent(X)
            for l in o.labels:
                fb *= extent(rng[l])
            fl += fb
    outl = [l for l in labs if l in keep]
    sz = 1.0
    for l in outl:
        sz *= extent(rng[l])
    return fl, sz, outl


def greedy_tree(ops, ext, rng, cap=2.5e9):
    """Cheapest binary contraction tree (exhaustive for up to 6 operands, greedy beyond).

    Returns (steps, flops, result operand); steps are (a, b, new) in execution order.
    Intermediates larger than `cap` elements are avoided when possible.
    """
    ops = list(ops)
    if len(ops) <= 6:
        best = _search(tuple(ops), frozenset(ext), rng, cap, {})
        return list(best[2]), best[1], best[3]
    steps = []
    total = 0.0
    while len(ops) > 1:
        best = None
        for i, j in itertools.combinations(range(len(ops)), 2):
            others = set(ext)
            for k, o in enumerate(ops):
                if k not in (i, j):
                    others |= set(o.labels)
            fl, sz, outl = _pair_cost(ops[i], ops[j], others, rng)
            shared = set(ops[i].labels) & set(ops[j].labels)
            pen = 0 if shared else 1
            key = (pen, sz > cap, fl, sz)
            if best is None or key < best[0]:
                best = (key, i, j, outl)
        _, i, j, outl = best
        total += best[0][2]
        new = _new_operand(ops[i], ops[j], outl, rng)
        steps.append((ops[i], ops[j], new))
        ops = [o for k, o in enumerate(ops) if k not in (i, j)] + [new]
    return steps, total, ops[0]


def _new_operand(a, b, outl, rng):
    outl = sorted(outl, key=lambda l: (l not in a.labels,
                                       a.labels.index(l) if l in a.labels else b.labels.index(l)))
    return Operand("?", [rng[l] for l in outl], outl)


def _search(ops, ext, rng, cap, memo):
    """(penalty, flops, steps, result) of the cheapest tree over the operand tuple."""
    if len(ops) == 1:
        return (0, 0.0, (), ops[0])
    best = None
    n = len(ops)
    for i, j in itertools.combinations(range(n), 2):
        others = set(ext)
        for k, o in enumerate(ops):
            if k not in (i, j):
                others |= set(o.labels)
        fl, sz, outl = _pair_cost(ops[i], ops[j], others, rng)
        shared = set(ops[i].labels) & set(ops[j].labels)
        pen = (0 if shared else 1) + (1 if sz > cap else 0)
        new = _new_operand(ops[i], ops[j], outl, rng)
        rest = tuple(o for k, o in enumerate(ops) if k not in (i, j)) + (new,)
        sub = _search(rest, ext, rng, cap, memo)
        cand = (pen + sub[0], 2.0 * fl + sub[1], ((ops[i], ops[j], new),) + sub[2], sub[3])
        if best is None or cand[:2] < best[:2]:
            best = cand
    return best


def _is_ladder(ops, ext, rng):
    """B(X,c,e) B(X,d,f) with c,d,e,f particle-type, c,d = ext[2],ext[3], e,f internal."""
    bs = [o for o in ops if o.name == "B"]
    if len(bs) != 2 or len(ext) != 4:
        return None
    b1, b2 = bs
    if b1.labels[0] != b2.labels[0]:
        return None
    if any(parent(r) != P for r in b1.ranges[1:] + b2.ranges[1:]):
        return None
    k, l, c, d = ext
    for x, y in ((b1, b2), (b2, b1)):
        if c in x.labels[1:] and d in y.labels[1:]:
            e = x.labels[1] if x.labels[2] == c else x.labels[2]
            f = y.labels[1] if y.labels[2] == d else y.labels[2]
            if e in ext or f in ext or e == c or f == d:
                return None
            if rng[c] != P or rng[d] != P:
                return None
            rest = [o for o in ops if o is not b1 and o is not b2]
            labs = set()
            for o in rest:
                labs |= set(o.labels)
            if labs != {k, l, e, f}:
                return None
            return rest, (k, l, e, f)
    return None


class _Terms:
    """Terms of one plan section, sorted into the emission strategies."""

    def __init__(self):
        self.groups = OrderedDict()     # sum-before-contract groups
        self.dfterms = []               # terms with an integral over >= 3 particle indices
        self.direct = []
        self.ladder = []                # (coef, rest, (k, l, e, f), rng): R2 += (ce|df) rest[k,l,e,f]

    def add_sf(self, t: SFTerm, target, out_ranges, allow_ladder=True):
        ops = factor_operands(t)
        rng = _rng_of(ops, t.ext, out_ranges)
        if target == "R2" and allow_ladder:
            lad = _is_ladder(ops, t.ext, rng)
            if lad is not None:
                self.ladder.append((t.coef, lad[0], lad[1], rng))
                return
        self.add_ops(target, t.coef, t.ext, out_ranges, ops, rng)

    def add_ops(self, target, coef, ext, out_ranges, ops, rng):
        ext = tuple(ext)
        bs = [o for o in ops if o.name == "B"]
        if len(bs) == 2:
            self.dfterms.append((target, coef, ext, out_ranges, ops, rng))
            return
        if len(ops) == 1:
            self.direct.append((target, coef, ext, out_ranges, ops, rng))
            return
        # sum-before-contract: the last contraction pairs one stored operand P0 with an
        # intermediate Y of the others; pick the P0 with the cheapest total, preferring T2
        _, gflops, _ = greedy_tree(ops, ext, rng)
        choice = None
        for big in range(len(ops)):
            if ops[big].size() < 1e6:
                continue
            rest = [o for i, o in enumerate(ops) if i != big]
            keep = set(ext) | set(ops[big].labels)
            if len(rest) == 1:
                ys, yf, Yo = [], 0.0, rest[0]
            else:
                ys, yf, Yo = greedy_tree(rest, keep, rng)
            fl_last, _, _ = _pair_cost(ops[big], Yo, set(ext), rng)
            cost = yf + 2.0 * fl_last
            pref = 0 if ops[big].name in ("T2", "XL", "YL") else 1
            cand = (cost > 1.5 * gflops + 1e6, pref, cost)
            if choice is None or cand < choice[0]:
                choice = (cand, big, ys, yf, Yo)
        if choice is not None and not choice[0][0]:
            _, big, ysteps, yflops, Yop = choice
            P0 = ops[big]
            ren = {}
            for i, l in enumerate(ext):
                ren[l] = f"o{i}"
            cnt = 0
            for l in P0.labels:
                if l not in ren:
                    ren[l] = f"c{cnt}"
                    cnt += 1
            ylabs = sorted(Yop.labels, key=lambda l: ren[l])
            # group on parent ranges: every label except the outputs carried by P0 is
            # widened to H or P; members fill sub-blocks of the shared intermediate
            p0_ext = set(P0.labels) & set(ext)
            g_rng = {l: (rng[l] if l in p0_ext else _widen(rng[l])) for l in rng}
            key = (target, P0.name, tuple(g_rng[l] for l in P0.labels), tuple(ren[l] for l in P0.labels),
                   tuple(g_rng[l] for l in ext), tuple((ren[l], g_rng[l]) for l in ylabs))
            self.groups.setdefault(key, []).append((coef, ysteps, Yop, ylabs, P0, ext, out_ranges, rng, ren, g_rng))
        else:
            self.direct.append((target, coef, ext, out_ranges, ops, rng))

    def emit(self, plan):
        _emit_groups(plan, self.groups)
        _emit_df_terms(plan, self.dfterms)
        _emit_direct(plan, self.direct)


def _emit_tau(plan, ladder):
    """tau = sum of the ladder terms' amplitude products, then tau + tau^T(pairs)."""
    plan.lines.append("ALLOC TAU HHPP")
    plan.lines.append("ZERO TAU")
    for coef, rest, (k, l, e, f), rng in ladder:
        out = Operand("TAU", (rng[k], rng[l], rng[e], rng[f]), (k, l, e, f))
        _emit_into(plan, coef, rest, out, rng)
    plan.lines.append("SYMMETRIZE TAU")


def _emit_residual(plan, name, r1_terms, s2_terms):
    """One residual section: the non-ladder terms into R1 and S2, R2 = S2 + S2^T(pairs), then the
    ladder (tau accumulated and symmetrized over pairs, contracted with (ce|df) built from B).
    The ladder block runs from ALLOC TAU to FREE TAU.  Returns the section's ladder terms."""
    res = _Terms()
    for t in r1_terms:
        res.add_sf(t, "R1", (t.rng[t.ext[0]], t.rng[t.ext[1]]))
    for t in s2_terms:
        res.add_sf(t, "R2", tuple(t.rng[l] for l in t.ext))
    plan.lines.append(f"SECTION {name}")
    plan.lines.append("ZERO R1")
    plan.lines.append("ZERO R2")
    res.emit(plan)
    plan.lines.append("SYMMETRIZE R2")
    if res.ladder:
        _emit_tau(plan, res.ladder)
        plan.lines.append("LADDER R2 TAU")
        nP, nH, nx = extent(P), extent(H), extent(X)
        plan.ladder_flops = nP * nP * (nP + 1) / 2 * nP * nx * 2 + nH * nH * nP * (nP + 1) / 2 * nP * nP * 2
        plan.flops += plan.ladder_flops
        plan.lines.append("FREE TAU")
    plan.lines.append("MASK R1 R2")
    plan.lines.append("END")
    return res.ladder


def compile_plan(e_terms, r1_terms, s2_terms, adjoint=True, groups=None):
    """groups: optional {"lin": (r1, s2), "quad": (r1, s2)}, compiled into the sections
    residual_lin and residual_quad (the term groups a caller may evaluate on their own)."""
    plan = Plan()
    ladder = _emit_residual(plan, "residual", r1_terms, s2_terms)
    res_flops = plan.flops
    if groups is not None:
        for g in ("lin", "quad"):
            f0, l0 = plan.flops, plan.ladder_flops
            _emit_residual(plan, f"residual_{g}", *groups[g])
            plan.flops, plan.ladder_flops = f0, l0
    # energy: every term is a full contraction
    plan.lines.append("SECTION energy")
    plan.lines.append("ZERO E")
    en = _Terms()
    for t in e_terms:
        en.add_sf(t, "E", ())
    en.emit(plan)
    plan.lines.append("END")
    if adjoint:
        compile_adjoint(plan, e_terms, r1_terms, s2_terms, ladder)
    return plan, res_flops


# ---- adjoint sections -----------------------------------------------------------------------
#
# With x = (XR1, XL) the cotangents of the masked residuals (XL pair-symmetric), the
# residual section computes R1 = mask(S1), R2 = mask(S2 + S2^T + W.(tau + tau^T)),
# W[c,d,e,f] = (ce|df).  Its vector-Jacobian products:
#   cotangent of S1 = XR1;  of S2 = 2 XL;  of tau = 2 YL with YL = W.XL (the ladder applied to XL);
#   dB from the ladder: 2 sum_{d,f} V[c,e,d,f] B[X,d,f], V[c,e,d,f] = sum_kl XL[k,l,c,d] tau_s[k,l,e,f].
# Each term coef * prod(ops) of a section contributes, for every differentiable operand o,
#   d<o>[o.labels] += coef * (cotangent) * prod(other operands),
# compiled with the same strategies as the forward terms.  Stored integral blocks
# I = sum_X B B collect dI first, and dI is contracted with B at the end of a section.

_GRAD = {"T1": "dT1", "T2": "dT2", "f": "dF", "B": "dB", "I4": "dI4", "I3": "dI3", "IJ": "dIJ", "IK": "dIK"}
_AMPS = ("T1", "T2")
_THETA = ("f", "B", "I4", "I3", "IJ", "IK")
_IBLOCKS = {"I4": (H, H, H, H), "I3": (H, H, H, P), "IJ": (H, H, P, P), "IK": (H, P, H, P)}


def _derivatives(terms: _Terms, target, coef, ext, out_ranges, ops, rng, cot, wrt):
    for i, o in enumerate(ops):
        if o.name not in wrt:
            continue
        if len(set(o.labels)) != len(o.labels):
            raise ValueError(f"repeated label in a differentiated operand {o.text()}")
        rest = ([cot] if cot is not None else []) + [x for j, x in enumerate(ops) if j != i]
        if not rest:
            raise ValueError("constant derivative term")
        terms.add_ops(_GRAD[o.name], coef, o.labels, o.ranges, rest, rng)


def _cotangent(target, ext, rng):
    if target == "R1":
        return Operand("XR1", [rng[l] for l in ext], ext), 1
    if target == "R2":
        return Operand("XL", [rng[l] for l in ext], ext), 2
    return None, 1


def _emit_dI_to_dB(plan):
    """dB[X,p,r] += sum_qs dI[p,r,q,s] B[X,q,s] and dB[X,q,s] += sum_pr dI[p,r,q,s] B[X,p,r]."""
    for name, (r0, r1, r2, r3) in _IBLOCKS.items():
        d = Operand("d" + name, (r0, r1, r2, r3), ("0", "1", "2", "3"))
        plan.contract(Operand("dB", (X, r0, r1), ("X0", "0", "1")), 1, d, Operand("B", (X, r2, r3), ("X0", "2", "3")))
        plan.contract(Operand("dB", (X, r2, r3), ("X0", "2", "3")), 1, d, Operand("B", (X, r0, r1), ("X0", "0", "1")))


def compile_adjoint(plan, e_terms, r1_terms, s2_terms, ladder):
    # d/dT of <x, r>: the products J_r^T x used by the Lagrangian iteration
    tt = _Terms()
    for target, terms in (("R1", r1_terms), ("R2", s2_terms)):
        for t in terms:
            ops = factor_operands(t)
            out_ranges = tuple(t.rng[l] for l in t.ext)
            rng = _rng_of(ops, t.ext, out_ranges)
            if target == "R2" and _is_ladder(ops, t.ext, rng) is not None:
                continue
            cot, w = _cotangent(target, t.ext, rng)
            _derivatives(tt, target, t.coef * w, t.ext, out_ranges, ops, rng, cot, _AMPS)
    for coef, rest, (k, l, e, f), rng in ladder:
        if any(o.name not in _AMPS for o in rest):
            raise ValueError("ladder amplitude products must hold amplitudes only")
        cot = Operand("YL", (rng[k], rng[l], rng[e], rng[f]), (k, l, e, f))
        _derivatives(tt, "R2", coef * 2, (k, l, e, f), None, rest, rng, cot, _AMPS)
    plan.lines.append("SECTION adjoint_t")
    plan.lines.append("ZERO dT1")
    plan.lines.append("ZERO dT2")
    if ladder:
        plan.lines.append("ALLOC YL HHPP")
        plan.lines.append("ZERO YL")
        plan.lines.append("LADDER YL XL")
    tt.emit(plan)
    if ladder:
        plan.lines.append("FREE YL")
    plan.lines.append("SYMHALF dT2")
    plan.lines.append("MASK dT1 dT2")
    plan.lines.append("END")

    # d/d(f, B) of <x, r>
    th = _Terms()
    for target, terms in (("R1", r1_terms), ("R2", s2_terms)):
        for t in terms:
            ops = factor_operands(t)
            out_ranges = tuple(t.rng[l] for l in t.ext)
            rng = _rng_of(ops, t.ext, out_ranges)
            if target == "R2" and _is_ladder(ops, t.ext, rng) is not None:
                continue
            cot, w = _cotangent(target, t.ext, rng)
            _derivatives(th, target, t.coef * w, t.ext, out_ranges, ops, rng, cot, _THETA)
    plan.lines.append("SECTION adjoint_theta")
    plan.lines.append("ZERO dF")
    plan.lines.append("ZERO dB")
    for name, rr in _IBLOCKS.items():
        plan.lines.append(f"ALLOC d{name} {''.join(RN[r] for r in rr)}")
        plan.lines.append(f"ZERO d{name}")
    th.emit(plan)
    if ladder:
        _emit_tau(plan, ladder)
        plan.lines.append("LADDERGRAD dB XL TAU")
        plan.lines.append("FREE TAU")
    _emit_dI_to_dB(plan)
    for name in _IBLOCKS:
        plan.lines.append(f"FREE d{name}")
    plan.lines.append("END")

    # gradient of the energy functional with respect to T, f and B
    eg = _Terms()
    for t in e_terms:
        ops = factor_operands(t)
        rng = _rng_of(ops, t.ext, ())
        _derivatives(eg, "E", t.coef, (), (), ops, rng, None, _AMPS + _THETA)
    plan.lines.append("SECTION energy_grad")
    for name in ("dT1", "dT2", "dF", "dB"):
        plan.lines.append(f"ZERO {name}")
    for name, rr in _IBLOCKS.items():
        plan.lines.append(f"ALLOC d{name} {''.join(RN[r] for r in rr)}")
        plan.lines.append(f"ZERO d{name}")
    eg.emit(plan)
    _emit_dI_to_dB(plan)
    for name in _IBLOCKS:
        plan.lines.append(f"FREE d{name}")
    plan.lines.append("SYMHALF dT2")
    plan.lines.append("MASK dT1 dT2")
    plan.lines.append("END")


def _emit_steps(plan, steps, final_out=None, alpha=1):
    """Emit contractions of a tree; the last one goes into final_out (accumulate) if given.

    Returns the mapping id(tree node) -> emitted operand for intermediates kept alive
    (only when final_out is None: the caller frees them).
    """
    names = {}
    for idx, (a, b, new) in enumerate(steps):
        a = names.get(id(a), a)
        b = names.get(id(b), b)
        last = idx == len(steps) - 1
        if last and final_out is not None:
            _emit_pair(plan, final_out, alpha, a, b, fresh=False)
        else:
            nm = plan.new_tmp(new.ranges)
            o = Operand(nm, new.ranges, new.labels)
            _emit_pair(plan, o, 1, a, b, fresh=True)
            names[id(new)] = o
        for x in (a, b):
            if x.name.startswith("t") and x.name[1:].isdigit():
                plan.free(x.name)
    return names


def _emit_pair(plan, out, alpha, a, b, fresh):
    if a.name == "ERI" or b.name == "ERI":
        eri, y = (a, b) if a.name == "ERI" else (b, a)
        rng = {}
        for o in (out, eri, y):
            for l, r in zip(o.labels, o.ranges):
                rng[l] = r
        if fresh:
            plan.lines.append(f"ZERO {out.name}")
        _emit_dfc(plan, alpha, out, eri.src[0], eri.src[1], eri.labels, y, rng)
    else:
        plan.contract(out, alpha, a, b, fresh=fresh)


def _emit_into(plan, coef, ops, out, rng):
    if len(ops) == 1:
        plan.add(out, coef, ops[0])
        return
    steps, _, _ = greedy_tree(ops, set(out.labels), rng)
    _emit_steps(plan, steps, final_out=out, alpha=coef)


ACC_CAP = 2.5e9   # elements (cost-model size) above which a group accumulator is chunked
PRECOMBINE = True  # sum permuted views of a stored operand before the product they share
SUM_FLOP_PER_BYTE = 20.0  # flops a product must save per byte the summation of its operands moves


def _vol(ranges):
    n = 1.0
    for r in ranges:
        n *= extent(r)
    return n


def _chunk_role(members, ylabs0, ext0, g0, ren0):
    """Canonical role of a label of the group's accumulator that every member's block
    covers over the group's full range, so the group can run per chunk of it (an output
    label of the final contraction, or one it sums over with the stored operand)."""
    best = None
    for l in ylabs0:
        role, r0 = ren0[l], g0[l]
        ok = True
        for m in members:
            ylabs, rng, ren = m[3], m[7], m[8]
            lm = [x for x in ylabs if ren.get(x) == role]
            if len(lm) != 1 or rng[lm[0]] != r0:
                ok = False
                break
        if ok and (best is None or extent(r0) > extent(best[1])):
            best = (role, r0)
    return None if best is None else best[0]


_VALID = (C, A, V, H, P, G, X)


def _tight_ranges(members):
    """Per label role of a group, the union of the ranges its members use: the accumulator,
    the stored operand's summed labels and the outputs carried by the accumulator span only
    the sub-blocks some member writes (instead of the whole hole or particle range)."""
    tight = {}
    for m in members:
        rngm, renm = m[7], m[8]
        for l, role in renm.items():
            tight[role] = tight.get(role, 0) | rngm[l]
    return tight



def _stored(o):
    """An operand that holds a stored tensor (not an intermediate of this plan, not a DF term)."""
    return not (o.name in ("?", "ERI") or (o.name.startswith("t") and o.name[1:].isdigit()))


def _canon(op, out_labels, own=None):
    """Labels of op named relative to the output: output label i -> 'o<i>'; a summed label by
    its order of appearance in the operand that defines `own` (created here when None)."""
    pos = {l: i for i, l in enumerate(out_labels)}
    make = own is None
    own = {} if make else own
    c = []
    for l in op.labels:
        if l in pos:
            c.append(f"o{pos[l]}")
        else:
            if l not in own:
                if not make:
                    return None, own
                own[l] = f"s{len(own)}"
            c.append(own[l])
    return tuple(c), own


def _sum_views(plan, terms, names, ranges):
    """A new intermediate sum c * view over terms (c, operand, {canonical name: label}), with its
    labels in canonical order `names` over `ranges`."""
    tmp = plan.new_tmp(ranges)
    plan.lines.append(f"ZERO {tmp}")
    for c, op, inv in terms:
        plan.add(Operand(tmp, ranges, [inv[n] for n in names]), c, op)
    return tmp


def _emit_summed_products(plan, items):
    """out += coef * a . b for items (coef, out, a, b) of stored a, b and one output.

    Products that share one operand (the same stored tensor in the same pattern relative to
    the output) are emitted once, the other operands (views of one stored tensor) summed
    first.  When the partner sums of all groups are proportional (after matching their summed
    labels), the shared operands are summed too and one product remains:
    sum_g lam_g X_g . P = (sum_g lam_g X_g) . P."""
    best = None
    for side in (0, 1):
        groups = OrderedDict()
        ok = True
        for coef, out, a, b in items:
            X, Z = (a, b) if side == 0 else (b, a)
            cx, own = _canon(X, out.labels)
            cz, _ = _canon(Z, out.labels, own)
            if cz is None:
                ok = False
                break
            key = (X.name, cx, X.ranges, out.ranges, Z.name, tuple(sorted(cz)))
            g = groups.setdefault(key, OrderedDict())
            zk = (cz, Z.ranges)
            if zk in g:
                g[zk][0] += coef
                g[zk][2].append((coef, out, a, b))
            else:
                g[zk] = [coef, (out, X, Z, own), [(coef, out, a, b)]]
        if ok and (best is None or len(groups) < len(best[1])):
            best = (side, groups)
    if best is None or len(best[1]) == len(items):
        for coef, out, a, b in items:
            plan.contract(out, coef, a, b)
        return
    groups = [(k, g) for k, g in best[1].items() if any(v[0] != 0 for v in g.values())]

    def product_flops(out, X, Z):
        rng = {}
        for o in (out, X, Z):
            for l, r in zip(o.labels, o.ranges):
                rng[l] = r
        f = 2.0
        for r in rng.values():
            f *= extent(r)
        return f

    def worth(saved_flops, sums):
        """A sum of n views of size s moves (24 n + 8) s bytes (zero, then read each view and
        read-modify-write the sum); it pays when the products it saves take longer."""
        moved = sum((24.0 * n + 8.0) * size for n, size in sums)
        return saved_flops > SUM_FLOP_PER_BYTE * moved

    def inverse(out, own):
        inv = {f"o{i}": l for i, l in enumerate(out.labels)}
        inv.update({n: l for l, n in own.items()})
        return inv

    def partner_sum(g, rename):
        """Intermediate sum of a group's partners; returns (tmp, names, ranges) with names in the
        renamed canonical naming."""
        zks = list(g.keys())
        names = sorted(rename.get(n, n) for n in zks[0][0])
        rmap = {rename.get(n, n): r for n, r in zip(zks[0][0], zks[0][1])}
        ranges = [rmap[n] for n in names]
        terms = []
        for zk in zks:
            c, (out, X, Z, own) = g[zk][:2]
            inv = inverse(out, own)
            back = {rename.get(n, n): inv[n] for n in inv}
            terms.append((c, Z, back))
        return _sum_views(plan, terms, names, ranges), names, ranges

    # proportional partner sums: match each group's summed-label names to the first group's
    merge = None
    if len(groups) > 1 and len({(k[0], tuple(sorted(k[1])), k[3], k[4]) for k, _ in groups}) == 1:
        k0, g0 = groups[0]
        base = {zk: v[0] for zk, v in g0.items()}
        snames = sorted(n for n in k0[1] if n.startswith("s"))
        merge = [(k0, g0, {}, 1.0)]
        for k, g in groups[1:]:
            found = None
            for perm in itertools.permutations(snames):
                rn = dict(zip(snames, perm))
                mapped = {}
                for (cz, zr), v in g.items():
                    mapped[(tuple(rn.get(n, n) for n in cz), zr)] = v[0]
                if set(mapped) != set(base):
                    continue
                j = next(zk for zk in base if base[zk] != 0)
                lam = mapped[j] / base[j]
                if all(abs(mapped[zk] - lam * base[zk]) <= 1e-12 * max(1.0, abs(mapped[zk])) for zk in base):
                    xr0 = dict(zip(k0[1], k0[2]))
                    xr = {rn.get(n, n): r for n, r in zip(k[1], k[2])}
                    if xr == xr0:
                        found = (rn, lam)
                        break
            if found is None:
                merge = None
                break
            merge.append((k, g, found[0], found[1]))
    if merge is not None:
        k0, g0 = groups[0]
        out0, X0, Z0, own0 = next(iter(g0.values()))[1]
        nprod = sum(len(g) for _, g in groups)
        if not worth((nprod - 1) * product_flops(out0, X0, Z0), [(len(merge), X0.size()), (len(g0), Z0.size())]):
            merge = None
    if merge is not None:
        k0, g0 = groups[0]
        xnames = sorted(k0[1])
        xrm = dict(zip(k0[1], k0[2]))
        xr = [xrm[n] for n in xnames]
        xterms = []
        for k, g, rn, lam in merge:
            out, X, Z, own = next(iter(g.values()))[1]
            inv = inverse(out, own)
            back = {rn.get(n, n): inv[n] for n in inv}
            xterms.append((lam, X, back))
        xt = _sum_views(plan, xterms, xnames, xr)
        zt, znames, zr = partner_sum(g0, {})
        out0, X0, Z0, own0 = next(iter(g0.values()))[1]
        inv0 = inverse(out0, own0)
        plan.contract(out0, 1, Operand(xt, xr, [inv0[n] for n in xnames]), Operand(zt, zr, [inv0[n] for n in znames]))
        plan.free(zt)
        plan.free(xt)
        return
    for k, g in groups:
        zks = list(g.keys())
        out0, X0, Z0, own0 = g[zks[0]][1]
        if len(zks) == 1 or not worth((len(zks) - 1) * product_flops(out0, X0, Z0), [(len(zks), Z0.size())]):
            # the products as they were, each with its own output labels and operand order
            for zk in zks:
                for c, out, a, b in g[zk][2]:
                    plan.contract(out, c, a, b)
            continue
        zt, znames, zr = partner_sum(g, {})
        out0, X0, Z0, own0 = g[zks[0]][1]
        inv0 = inverse(out0, own0)
        plan.contract(out0, 1, X0, Operand(zt, zr, [inv0[n] for n in znames]))
        plan.free(zt)


def _emit_groups(plan, groups):
    for key, members in groups.items():
        target = key[0]
        coef0, ysteps0, Yop0, ylabs0, P00, ext0, out_ranges0, rng0, ren0, g0w = members[0]
        if len(members) == 1 and not ysteps0:
            # plain product of two stored tensors
            out = Operand(target, out_ranges0, ext0)
            plan.contract(out, coef0, P00, Yop0)
            continue
        tight = _tight_ranges(members)
        g0 = {l: (tight[ren0[l]] if l in ren0 and tight.get(ren0[l]) in _VALID else r) for l, r in g0w.items()}
        # an accumulator too large to hold whole is built and consumed in chunks of an
        # output label that every member covers over the same range (leading dimension)
        chunk = None
        if _vol([g0[l] for l in ylabs0]) > ACC_CAP:
            chunk = _chunk_role(members, ylabs0, ext0, g0, ren0)

        def order(ylabs, ren):
            if chunk is None:
                return list(ylabs)
            return [l for l in ylabs if ren.get(l) == chunk] + [l for l in ylabs if ren.get(l) != chunk]

        ylabs0 = order(ylabs0, ren0)
        yr = [g0[l] for l in ylabs0]
        if chunk is not None:
            plan.lines.append(f"LOOP t{plan.tmp} 0")
        acc = plan.new_tmp(yr)
        plan.lines.append(f"ZERO {acc}")
        # second level: members whose intermediate is one product X * Z of two stored
        # tensors with the same X pattern share X; their Z's are summed first
        sub = OrderedDict()
        rest_members = []
        def is_tmp(o):
            return o.name == "?" or (o.name.startswith("t") and o.name[1:].isdigit())

        for m in members:
            coef, ysteps, Yop, ylabs, P0m, ext, out_ranges, rng, ren, g = m
            if ysteps:
                # the member's intermediate is X * Z with X stored; Z is stored too (one step) or
                # computed by the member's earlier steps (the prefix), which then accumulate it
                a, b, new = ysteps[-1]
                prefix = ysteps[:-1]
                placed = False
                for X, Z in ((a, b), (b, a)):
                    if is_tmp(X) or (is_tmp(Z) if not prefix else Z.name != "?"):
                        continue
                    # roles: labels of Y map to their canonical names in the group
                    yrole = {l: ren.get(l, None) for l in ylabs}
                    inner = [l for l in X.labels if l in Z.labels]
                    iren = {l: f"i{k}" for k, l in enumerate(inner)}
                    # X keeps the exact ranges of its own Y labels; inner labels widen
                    xkey = tuple((yrole.get(l) or iren[l], _widen(rng[l]) if l in iren else rng[l])
                                 for l in X.labels)
                    zlabs = sorted(Z.labels, key=lambda l: (yrole.get(l) or iren[l]))
                    zkey = tuple((yrole.get(l) or iren[l], _widen(rng[l])) for l in zlabs)
                    key2 = (X.name, xkey, zkey)
                    sub.setdefault(key2, []).append((coef, X, Z, zlabs, rng, ylabs, m, prefix))
                    placed = True
                    break
                if placed:
                    continue
            rest_members.append(m)
        for key2, items in sub.items():
            if len(items) == 1:
                rest_members.append(items[0][6])
                continue
            coef0_, X0, Z0, zl0, rng0_, yl0, m0, _ = items[0]
            yl0 = order(yl0, m0[8])
            # Z's ranges: the union of the items' own ranges, position by position
            zt = [0] * len(zl0)
            for it in items:
                for i, l in enumerate(it[3]):
                    zt[i] |= it[4][l]
            zr = [r if r in _VALID else _widen(rng0_[l]) for r, l in zip(zt, zl0)]
            zpos = {l: i for i, l in enumerate(zl0)}
            zacc = plan.new_tmp(zr)
            plan.lines.append(f"ZERO {zacc}")
            single = []
            for coef, X, Z, zlabs, rng, ylabs, m, prefix in items:
                zop = Operand(zacc, [rng[l] for l in zlabs], zlabs)
                if prefix and len(prefix) == 1 and chunk is None and PRECOMBINE and \
                        _stored(prefix[0][0]) and _stored(prefix[0][1]):
                    single.append((coef, zop, prefix[0][0], prefix[0][1]))
                elif prefix:
                    _emit_steps(plan, prefix, final_out=zop, alpha=coef)
                else:
                    plan.add(zop, coef, Z)
            if single:
                _emit_summed_products(plan, single)
            # X over the ranges of the first member, its inner labels over Z's ranges
            xr = [(zr[zpos[l]] if (l in zl0 and l not in yl0) else r) for l, r in zip(X0.labels, X0.ranges)]
            Xop = Operand(X0.name, xr, X0.labels)
            accop = Operand(acc, [(rng0_[l] if l in X0.labels else zr[zpos[l]]) for l in yl0], yl0)
            plan.contract(accop, 1, Xop, Operand(zacc, zr, zl0))
            plan.free(zacc)
        single = []
        for coef, ysteps, Yop, ylabs, P0m, ext, out_ranges, rng, ren, g in rest_members:
            # the member's own (possibly narrower) ranges address a sub-block of acc
            ylabs = order(ylabs, ren)
            accop = Operand(acc, [rng[l] for l in ylabs], ylabs)
            if not ysteps:
                plan.add(accop, coef, Yop)
            elif len(ysteps) == 1 and chunk is None and PRECOMBINE and _stored(ysteps[0][0]) and \
                    _stored(ysteps[0][1]):
                single.append((coef, accop, ysteps[0][0], ysteps[0][1]))
            else:
                _emit_steps(plan, ysteps, final_out=accop, alpha=coef)
        if single:
            _emit_summed_products(plan, single)
        out = Operand(target, [g0[l] for l in ext0], ext0)
        P0 = Operand(P00.name, [g0[l] for l in P00.labels], P00.labels)
        plan.contract(out, 1, P0, Operand(acc, yr, ylabs0))
        plan.free(acc)
        if chunk is not None:
            plan.lines.append("ENDLOOP")


def _nbig(o):
    return sum(1 for r in o.ranges if r != X and parent(r) == P)


def _emit_df_terms(plan, dfterms):
    """Terms whose integral has three or more particle indices.

    1. A two-index factor (T1, gA, eA, f) that shares a particle index with one B
       factor and no index with the other is contracted into it first when that
       lowers the number of particle indices ("dressing").
    2. The integral (pr|qs) = sum_X L1[X,p,r] L2[X,q,s] then enters the tree
       search as one leaf: whichever operand it meets is contracted with it by a
       DFC operation that builds the integral block by block from L1, L2.
    Terms whose last step contracts the same integral pattern with the same
    intermediate pattern share one accumulated intermediate.
    """
    groups = OrderedDict()
    for target, coef, ext, out_ranges, ops, rng in dfterms:
        bs = [o for o in ops if o.name == "B"]
        rest = [o for o in ops if o.name != "B"]
        pre = []          # dressing steps (a, b, new)
        changed = True
        while changed:
            changed = False
            for i, b in enumerate(bs):
                other = bs[1 - i]
                for f in rest:
                    if len(f.labels) != 2:
                        continue
                    sh = set(f.labels) & set(b.labels[1:])
                    if not sh or set(f.labels) & set(other.labels[1:]):
                        continue
                    if any(set(f.labels) & set(g.labels) for g in rest if g is not f):
                        # the free index of f must stay outside the remaining factors
                        free = set(f.labels) - sh
                        if free & set().union(*[set(g.labels) for g in rest if g is not f]):
                            continue
                    outl = [b.labels[0]] + [l for l in b.labels[1:] if l not in sh] + \
                           [l for l in f.labels if l not in sh]
                    if len(outl) != 3:
                        continue
                    new = Operand("?", [rng[l] for l in outl], outl)
                    if _nbig(new) >= _nbig(b):
                        continue
                    pre.append((b, f, new))
                    bs[i] = new
                    rest = [g for g in rest if g is not f]
                    changed = True
                    break
                if changed:
                    break
        l1, l2 = bs
        if _nbig(l1) + _nbig(l2) <= 2:
            # small enough to form: ordinary tree over all operands
            allops = [l1, l2] + rest
            if len(allops) == 1:
                continue
            steps, _, _ = greedy_tree(allops, set(ext), rng)
            out = Operand(target, out_ranges, ext)
            names = _emit_steps(plan, pre, final_out=None) if pre else {}
            steps = [(names.get(id(a), a), names.get(id(b), b), n) for a, b, n in steps]
            _emit_steps(plan, steps, final_out=out, alpha=coef)
            continue
        eri_l = l1.labels[1:] + l2.labels[1:]
        eri = Operand("ERI", [rng[l] for l in eri_l], eri_l)
        eri.src = (l1, l2)
        steps, _, res = greedy_tree([eri] + rest, set(ext), rng)
        last_a, last_b, _ = steps[-1]
        if last_a is eri or last_b is eri:
            Yfinal = last_b if last_a is eri else last_a
            ysteps = steps[:-1]
            ren = {l: f"o{i}" for i, l in enumerate(ext)}
            cnt = 0
            for l in eri_l:
                if l not in ren:
                    ren[l] = f"c{cnt}"
                    cnt += 1
            ylabs = sorted(Yfinal.labels, key=lambda l: ren.get(l, "z"))
            key = (target, tuple(ren[l] for l in eri_l), tuple(rng[l] for l in eri_l),
                   tuple(out_ranges), tuple((ren.get(l), rng[l]) for l in ylabs),
                   tuple(_src_key(x, ren) for x in (l1, l2)))
            groups.setdefault(key, []).append((coef, pre, ysteps, Yfinal, ylabs, eri, ext, out_ranges, rng))
        else:
            names = _emit_steps(plan, pre, final_out=None) if pre else {}
            steps = [(names.get(id(a), a), names.get(id(b), b), n) for a, b, n in steps]
            out = Operand(target, out_ranges, ext)
            _emit_steps(plan, steps, final_out=out, alpha=coef)
    for key, members in groups.items():
        target = key[0]
        coef0, pre0, ysteps0, Y0, ylabs0, eri0, ext0, out_ranges0, rng0 = members[0]
        yr = [rng0[l] for l in ylabs0]
        acc = plan.new_tmp(yr)
        plan.lines.append(f"ZERO {acc}")
        for coef, pre, ysteps, Yf, ylabs, eri, ext, out_ranges, rng in members:
            accop = Operand(acc, [rng[l] for l in ylabs], ylabs)
            names = _emit_steps(plan, pre, final_out=None) if pre else {}
            if not ysteps:
                plan.add(accop, coef, names.get(id(Yf), Yf))
            else:
                ys = [(names.get(id(a), a), names.get(id(b), b), n) for a, b, n in ysteps]
                _emit_steps(plan, ys, final_out=accop, alpha=coef)
            for nm in names.values():
                pass
        # the (possibly dressed) DF factors of the first member define the integral
        names0 = {}
        l1, l2 = eri0.src
        out = Operand(target, out_ranges0, ext0)
        if pre0:
            names0 = _emit_steps(plan, pre0, final_out=None)
        l1 = names0.get(id(l1), l1)
        l2 = names0.get(id(l2), l2)
        _emit_dfc(plan, 1, out, l1, l2, eri0.labels, Operand(acc, yr, ylabs0), rng0)
        plan.free(acc)
        for o in (l1, l2):
            if o.name.startswith("t") and o.name[1:].isdigit():
                plan.free(o.name)


def _src_key(o, ren):
    return (o.name, o.ranges, tuple(ren.get(l, "x") for l in o.labels[1:]))


def _emit_dfc(plan, alpha, out, l1, l2, eri_labels, y, rng):
    labs = set(out.labels) | set(eri_labels) | set(y.labels)
    fl = 2.0
    for l in labs:
        fl *= extent(rng[l])
    fb = 2.0 * extent(X)
    for l in eri_labels:
        fb *= extent(rng[l])
    plan.flops += fl + fb
    plan.lines.append(f"DFC {_num(alpha)} {out.text()} {l1.text()} {l2.text()} {y.text()}")


def _emit_dfgroups(plan, dfgroups):
    for key, members in dfgroups.items():
        target = key[0]
        coef0, ysteps0, Yop0, ylabs0, eri0, ext0, out_ranges0, rng0 = members[0]
        yr = [rng0[l] for l in ylabs0]
        acc = plan.new_tmp(yr)
        plan.lines.append(f"ZERO {acc}")
        for coef, ysteps, Yop, ylabs, eri_l, ext, out_ranges, rng in members:
            accop = Operand(acc, [rng[l] for l in ylabs], ylabs)
            if not ysteps:
                plan.add(accop, coef, Yop)
            else:
                _emit_steps(plan, ysteps, final_out=accop, alpha=coef)
        out = Operand(target, out_ranges0, ext0)
        eri = Operand("ERI", [rng0[l] for l in eri0], eri0)
        labs = set(ext0) | set(eri0) | set(ylabs0)
        fl = 2.0
        for l in labs:
            fl *= extent(rng0[l])
        # building (pr|qs) from B: 2 * naux * prod(eri extents)
        fb = 2.0 * extent(X)
        for l in eri0:
            fb *= extent(rng0[l])
        plan.flops += fl + fb
        plan.lines.append(f"DFC 1/1 {out.text()} {eri.text()} {Operand(acc, yr, ylabs0).text()}")
        plan.free(acc)


def _emit_direct(plan, direct):
    for target, coef, ext, out_ranges, ops, rng in direct:
        out = Operand(target, out_ranges, ext)
        _emit_into(plan, coef, ops, out, rng)


def _emit_scalar(plan, coef, ops, rng):
    steps, _, _ = greedy_tree(ops, set(), rng)
    out = Operand("E", (), ())
    _emit_steps(plan, steps, final_out=out, alpha=coef)
