"""Generalized Wick theorem for products of normal-ordered spin-orbital operators.

TEST INFRASTRUCTURE (CPU oracle).  Only tests/, the smoke check and the CPU
baseline of the benchmark may use this package; the product library never does.

Follows Section 2.1 of the paper (generalized normal ordering with respect to a
multi-determinant reference): the product of two normal-ordered strings is the
sum over all contraction patterns whose every contraction touches both strings,
where a contraction is
  * a creator of the left string with an annihilator of the right string:
    gamma^p_q = <a^+_p a_q>            (core: delta, active: 1-RDM, virtual: 0)
  * an annihilator of the left string with a creator of the right string:
    eta^p_q = delta^p_q - gamma^p_q    (core: 0, active: 1-hole RDM, virtual: delta)
  * a k-body density cumulant lambda_k (k = 2, 3) over k creators and k
    annihilators taken from both strings (active orbitals only).
The sign of a pattern is the parity of the permutation that brings every
contracted group next to each other in canonical order, followed by the
uncontracted creators and annihilators in their original order.

Orbital spaces are bit masks: C (core), A (active), V (virtual); a leg of the
Hamiltonian starts as G = C|A|V and is narrowed by the contraction it enters.
String convention (Section 2.1): a^{p1..pk}_{q1..qk} = a^+_p1 .. a^+_pk a_qk .. a_q1.
Four-body cumulants are never generated: with the paper's filters on the
two-fold commutator they cannot occur in any kept term (counted in the header
of ricmrcc.py).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

C, A, V = 1, 2, 4
G = C | A | V
H = C | A
P = A | V
SPACE_NAME = {C: "c", A: "a", V: "v", G: "g", H: "h", P: "p"}

CRE, ANN = 1, -1


class Term:
    """coef * prod(factors) * {seq}, summed over every label.

    factors: tuple of (tensor name, tuple of labels)
    seq:     tuple of (kind, label), the normal-ordered string in sequence order
    space:   dict label -> space mask
    """
    __slots__ = ("coef", "factors", "seq", "space")

    def __init__(self, coef, factors, seq, space):
        self.coef = Fraction(coef)
        self.factors = tuple(factors)
        self.seq = tuple(seq)
        self.space = dict(space)

    @property
    def rank(self):
        return sum(1 for k, _ in self.seq if k == CRE)

    def upper(self):
        return [l for k, l in self.seq if k == CRE]

    def lower(self):
        # a^{U}_{L} = a^+_U1 .. a^+_Uk a_Lk .. a_L1  ->  L is the reversed annihilator sequence
        return [l for k, l in self.seq if k == ANN][::-1]

    def labels(self):
        s = set()
        for _, ls in self.factors:
            s.update(ls)
        for _, l in self.seq:
            s.add(l)
        return s

    def relabel(self, offset):
        m = {l: l + offset for l in self.labels()}
        return Term(self.coef,
                    [(n, tuple(m[x] for x in ls)) for n, ls in self.factors],
                    [(k, m[l]) for k, l in self.seq],
                    {m[l]: s for l, s in self.space.items()})

    def scaled(self, c):
        return Term(self.coef * c, self.factors, self.seq, self.space)

    def __repr__(self):
        f = " ".join(f"{n}({','.join(SPACE_NAME[self.space[l]] + str(l) for l in ls)})"
                     for n, ls in self.factors)
        u = ",".join(SPACE_NAME[self.space[l]] + str(l) for l in self.upper())
        lo = ",".join(SPACE_NAME[self.space[l]] + str(l) for l in self.lower())
        return f"{self.coef} {f} {{{u};{lo}}}"


def operator(name, upper, lower, spaces_up, spaces_lo, coef=1, start=0):
    """A single operator coef * sum name(upper+lower... as stored) {a^{upper}_{lower}}.

    The tensor is stored with the index order given by `order` = upper + lower;
    labels are start, start+1, ...
    """
    k = len(upper)
    labs_u = list(range(start, start + k))
    labs_l = list(range(start + k, start + 2 * k))
    space = {}
    for l, s in zip(labs_u, spaces_up):
        space[l] = s
    for l, s in zip(labs_l, spaces_lo):
        space[l] = s
    seq = [(CRE, l) for l in labs_u] + [(ANN, l) for l in labs_l[::-1]]
    return labs_u, labs_l, seq, space


def _parity(order):
    inv = 0
    n = len(order)
    for i in range(n):
        oi = order[i]
        for j in range(i + 1, n):
            if order[j] < oi:
                inv += 1
    return -1 if inv % 2 else 1


def _lambda_groups(ops, origin, space, nA):
    """All candidate cumulant groups (k, creator positions, annihilator positions), k = 2, 3."""
    cre = [i for i, (k, l) in enumerate(ops) if k == CRE and space[l] & A]
    ann = [i for i, (k, l) in enumerate(ops) if k == ANN and space[l] & A]
    groups = []
    for k in (2, 3):
        for cs in itertools.combinations(cre, k):
            for an in itertools.combinations(ann, k):
                pos = cs + an
                if any(p < nA for p in pos) and any(p >= nA for p in pos):
                    groups.append((k, cs, an))
    return groups


def _disjoint_group_sets(groups, max_groups=3):
    out = [()]

    def rec(start, used, chosen):
        for gi in range(start, len(groups)):
            k, cs, an = groups[gi]
            s = set(cs) | set(an)
            if s & used:
                continue
            c2 = chosen + (groups[gi],)
            out.append(c2)
            if len(c2) < max_groups:
                rec(gi + 1, used | s, c2)

    rec(0, set(), ())
    return out


def _pair_matchings(ops, space, a_pos, b_pos):
    """All sets of pairwise contractions between remaining A and B positions."""
    res = []

    def rec(idx, used_b, chosen):
        if idx == len(a_pos):
            res.append(tuple(chosen))
            return
        i = a_pos[idx]
        rec(idx + 1, used_b, chosen)
        ki, li = ops[i]
        for j in b_pos:
            if j in used_b:
                continue
            kj, lj = ops[j]
            if ki == kj:
                continue
            common = space[li] & space[lj]
            if ki == CRE:       # a^+ (left) a (right): gamma, core or active
                if not common & (C | A):
                    continue
            else:               # a (left) a^+ (right): eta, active or virtual
                if not common & (A | V):
                    continue
            rec(idx + 1, used_b | {j}, chosen + [(i, j)])

    rec(0, frozenset(), [])
    return res


def product(ta: Term, tb: Term, min_contr=1, max_rank=None, allow_lambda=True):
    """Generalized-Wick expansion of {ta}{tb}; returns a list of Terms.

    Labels of tb must not collide with labels of ta (use Term.relabel).
    """
    ops = list(ta.seq) + list(tb.seq)
    nA = len(ta.seq)
    n = len(ops)
    origin = [0] * nA + [1] * (n - nA)
    space = dict(ta.space)
    space.update(tb.space)
    groups = _lambda_groups(ops, origin, space, nA) if allow_lambda else []
    out = []
    for gset in _disjoint_group_sets(groups):
        used = set()
        for k, cs, an in gset:
            used.update(cs)
            used.update(an)
        a_pos = [i for i in range(nA) if i not in used]
        b_pos = [j for j in range(nA, n) if j not in used]
        for pairs in _pair_matchings(ops, space, a_pos, b_pos):
            ncontr = len(pairs) + len(gset)
            if ncontr < min_contr:
                continue
            cused = set(used)
            for i, j in pairs:
                cused.add(i)
                cused.add(j)
            unc = [i for i in range(n) if i not in cused]
            unc_c = [i for i in unc if ops[i][0] == CRE]
            unc_a = [i for i in unc if ops[i][0] == ANN]
            if max_rank is not None and len(unc_c) > max_rank:
                continue
            # sign
            order = []
            for i, j in pairs:
                order += [i, j]
            for k, cs, an in gset:
                order += list(cs) + list(an)
            order += unc_c + unc_a
            sign = _parity(order)
            new_seq = [ops[i] for i in unc_c] + [ops[i] for i in unc_a]
            # branches of every pairwise contraction
            options = []
            for i, j in pairs:
                li, lj = ops[i][1], ops[j][1]
                common = space[li] & space[lj]
                opts = []
                if ops[i][0] == CRE:
                    if common & C:
                        opts.append(("delta", C, li, lj))
                    if common & A:
                        opts.append(("g1", A, li, lj))          # gamma^{li}_{lj}
                else:
                    if common & A:
                        opts.append(("e1", A, lj, li))          # eta^{lj}_{li}
                    if common & V:
                        opts.append(("delta", V, li, lj))
                options.append(opts)
            lam_factors = []
            lam_labels = []
            for k, cs, an in gset:
                up = tuple(ops[i][1] for i in cs)
                lo = tuple(ops[i][1] for i in an)[::-1]
                lam_factors.append(("l%d" % k, up + lo))
                lam_labels.extend(up + lo)
            for choice in itertools.product(*options):
                sp = dict(space)
                ok = True
                for l in lam_labels:
                    sp[l] &= A
                    if not sp[l]:
                        ok = False
                        break
                if not ok:
                    continue
                rename = {}
                extra = []
                for kind, s, x, y in choice:
                    sp[x] &= s
                    sp[y] &= s
                    if not sp[x] or not sp[y]:
                        ok = False
                        break
                    if kind == "delta":
                        rename[y] = x
                    else:
                        extra.append((kind, (x, y)))
                if not ok:
                    continue
                facs = list(ta.factors) + list(tb.factors) + extra + lam_factors
                if rename:
                    facs = [(nm, tuple(rename.get(l, l) for l in ls)) for nm, ls in facs]
                    for y in rename:
                        sp.pop(y, None)
                out.append(Term(ta.coef * tb.coef * sign, facs, new_seq, sp))
    return out


def products(As, Bs, **kw):
    out = []
    for a in As:
        for b in Bs:
            off = (max(a.labels()) + 1 - min(b.labels())) if a.labels() and b.labels() else 0
            out.extend(product(a, b.relabel(off), **kw))
    return out


def commutator(As, Bs, max_rank=None, pair_filter=None):
    """[A, B] = {A}{B} - {B}{A}; patterns without contractions cancel and are skipped.

    pair_filter(a, b) -> bool may exclude pairs of terms (e.g. by amplitude class).
    """
    out = []
    for a in As:
        for b in Bs:
            if pair_filter is not None and not pair_filter(a, b):
                continue
            la, lb = a.labels(), b.labels()
            off = max(la) + 1 - min(lb)
            out.extend(product(a, b.relabel(off), min_contr=1, max_rank=max_rank))
            off2 = max(lb) + 1 - min(la)
            out.extend(t.scaled(-1) for t in product(b, a.relabel(off2), min_contr=1, max_rank=max_rank))
    return out


# --- canonical form for merging equal terms --------------------------------------------

# antisymmetric index groups of each tensor (positions within the label tuple)
ANTISYM = {
    "v": ((0, 1), (2, 3)),
    "t2": ((0, 1), (2, 3)),
    "l2": ((0, 1), (2, 3)),
    "l3": ((0, 1, 2), (3, 4, 5)),
}


def _perm_sign_sort(keys):
    """Stable sort permutation of keys and its parity."""
    idx = sorted(range(len(keys)), key=lambda i: keys[i])
    return idx, _parity(idx)


def canonical(term: Term):
    """(key, sign): equal keys denote the same summed operator term up to sign."""
    items = [(n, list(ls)) for n, ls in term.factors]
    ups = term.upper()
    los = term.lower()
    items.append(("~op", ups + los))
    sign = 1
    names = {}
    for _ in range(4):
        def lab_key(l):
            return (term.space[l], names.get(l, 10 ** 6))

        def fac_key(it):
            n, ls = it
            return (n, tuple(term.space[l] for l in ls), tuple(names.get(l, 10 ** 6) for l in ls))

        items.sort(key=fac_key)
        names = {}
        for n, ls in items:
            for l in ls:
                if l not in names:
                    names[l] = len(names)
        new_items = []
        for n, ls in items:
            ls = list(ls)
            if n == "~op":
                r = len(ls) // 2
                groups = (tuple(range(r)), tuple(range(r, 2 * r)))
            else:
                groups = ANTISYM.get(n, ())
            for grp in groups:
                keys = [lab_key(ls[p]) for p in grp]
                perm, sg = _perm_sign_sort(keys)
                sign *= sg
                vals = [ls[grp[p]] for p in perm]
                for p, v in zip(grp, vals):
                    ls[p] = v
            new_items.append((n, ls))
        items = new_items
    key = tuple((n, tuple((term.space[l], names[l]) for l in ls)) for n, ls in sorted(
        items, key=lambda it: (it[0], tuple(term.space[l] for l in it[1]), tuple(names[l] for l in it[1]))))
    return key, sign


def merge(terms):
    """Sum terms with equal canonical form; drop zeros."""
    acc = {}
    rep = {}
    for t in terms:
        key, sg = canonical(t)
        if key in acc:
            acc[key] += t.coef * sg
        else:
            acc[key] = t.coef * sg
            rep[key] = (t, sg)
    out = []
    for key, c in acc.items():
        if c != 0:
            t, sg = rep[key]
            out.append(Term(c * sg, t.factors, t.seq, t.space))
    return out
