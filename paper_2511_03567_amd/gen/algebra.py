"""Symbolic derivation of the spin-free RIC-MRCCSD working equations over hole/particle ranges.

Build-time tool of the library: it turns the definitions of Section 2 of the
paper into a list of spin-free tensor-contraction terms that the plan compiler
factorizes for the GPU.  Nothing here runs on the solve path.

Ranges are bit masks over the orbital spaces of Table 1: C (core), A (active),
V (virtual); H = C|A (holes), P = A|V (particles), G = C|A|V.  A Hamiltonian
leg starts on G and is restricted by the contraction it takes part in.

Generalized normal ordering (Section 2.1).  In a product {X}{Y} every
contraction joins legs of both strings:
  creator of X with annihilator of Y : gamma = delta on C, 1-RDM on A;
  annihilator of X with creator of Y : eta   = 1-hole RDM on A, delta on V;
  k creators and k annihilators (k = 2, 3, active legs from both strings):
                                       k-body density cumulant.
Over a whole hole range gamma is written delta_H - eta_A and over a whole
particle range eta is written delta_P - gamma_A, so the large ranges keep plain
index identities and only active-block corrections carry density factors.

Spin integration (Section 2.3): every spin-orbital tensor of the theory is a
singlet and is written as a sum of spatial tensors times products of spin
Kronecker deltas pairing its upper with its lower indices,
  f^p_q            = f[p,q] d(p,q)
  <pq||rs>         = (pr|qs) d(p,r)d(q,s) - (ps|qr) d(p,s)d(q,r)
  t^{cd}_{kl}      = T2[k,l,c,d] d(c,k)d(d,l) - T2[k,l,d,c] d(c,l)d(d,k)
  gamma^p_q        = (Gamma1/2)[p,q] d(p,q),   eta^p_q = (1 - Gamma1/2)[p,q] d(p,q)
  lambda^{pq}_{rs} = K2[p,q,r,s] d(p,r)d(q,s) - K2[p,q,s,r] d(p,s)d(q,r)
  lambda^{pqr}_{stu} = sum_pi sgn(pi) K3[p,q,r,pi(s,t,u)] prod d(upper_i, lower_pi(i))
The spin sum of a product then counts closed delta loops (factor 2 each) and
requires every open path to join external indices of equal spin.  K2 and K3
are the kernels of those expansions (pseudo-inverse of the loop-count map in the
group algebra of S_2 and S_3, applied to the spin-free cumulants).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field
from fractions import Fraction

C, A, V = 1, 2, 4
H = C | A
P = A | V
G = C | A | V
RANGE_NAME = {C: "C", A: "A", V: "V", H: "H", P: "P", G: "G"}
UP, LO = "u", "l"


@dataclass
class SOTerm:
    """coef * prod(tensors) * {a^{upper}_{lower}} with every label summed; spin-orbital."""
    coef: Fraction
    tensors: list            # [(name, (labels...))]
    upper: list              # creator labels in operator order
    lower: list              # annihilator labels: a^{u1..uk}_{l1..lk} = a+u1..a+uk a_lk..a_l1
    rng: dict                # label -> range mask
    has_l2: bool = False

    def rank(self):
        return len(self.upper)

    def sequence(self):
        return [(UP, l) for l in self.upper] + [(LO, l) for l in reversed(self.lower)]

    def labels(self):
        s = set(self.upper) | set(self.lower)
        for _, ls in self.tensors:
            s.update(ls)
        return s


def _sign_of(order):
    s = 1
    o = list(order)
    for i in range(len(o)):
        for j in range(len(o) - 1 - i):
            if o[j] > o[j + 1]:
                o[j], o[j + 1] = o[j + 1], o[j]
                s = -s
    return s


def _gamma_options(r):
    """Values of a creator(left)-annihilator(right) contraction on range r."""
    r &= H
    if r == H:
        return [(1, "delta", H), (-1, "eA", A)]
    if r == C:
        return [(1, "delta", C)]
    if r == A:
        return [(1, "gA", A)]
    return []


def _eta_options(r):
    """Values of an annihilator(left)-creator(right) contraction on range r."""
    r &= P
    if r == P:
        return [(1, "delta", P), (-1, "gA", A)]
    if r == V:
        return [(1, "delta", V)]
    if r == A:
        return [(1, "eA", A)]
    return []


def wick_product(x: SOTerm, y: SOTerm, max_rank=None):
    """All connected contraction patterns of {x}{y} (at least one contraction)."""
    seq = [(k, l, 0) for k, l in x.sequence()] + [(k, l, 1) for k, l in y.sequence()]
    rng = dict(x.rng)
    rng.update(y.rng)
    n = len(seq)
    nx = len(x.sequence())
    act = [i for i in range(n) if rng[seq[i][1]] & A]
    cre_a = [i for i in act if seq[i][0] == UP]
    ann_a = [i for i in act if seq[i][0] == LO]
    cum = []
    for k in (2, 3):
        for cs in itertools.combinations(cre_a, k):
            for an in itertools.combinations(ann_a, k):
                g = cs + an
                if min(g) < nx <= max(g):
                    cum.append((k, cs, an))
    # sets of disjoint cumulant groups
    sets = [[]]
    frontier = [([], set(), 0)]
    while frontier:
        nxt = []
        for chosen, used, start in frontier:
            for gi in range(start, len(cum)):
                g = cum[gi]
                s = set(g[1]) | set(g[2])
                if s & used:
                    continue
                c2 = chosen + [g]
                sets.append(c2)
                nxt.append((c2, used | s, gi + 1))
        frontier = nxt
    out = []
    for cset in sets:
        used = set()
        for _, cs, an in cset:
            used |= set(cs) | set(an)
        xs = [i for i in range(nx) if i not in used]
        ys = [j for j in range(nx, n) if j not in used]
        for pairs in _matchings(seq, rng, xs, ys):
            if not pairs and not cset:
                continue
            taken = set(used)
            for i, j in pairs:
                taken |= {i, j}
            free_up = [i for i in range(n) if i not in taken and seq[i][0] == UP]
            free_lo = [i for i in range(n) if i not in taken and seq[i][0] == LO]
            if max_rank is not None and len(free_up) > max_rank:
                continue
            order = []
            for i, j in pairs:
                order += [i, j]
            for _, cs, an in cset:
                order += list(cs) + list(an)
            order += free_up + free_lo
            sign = _sign_of(order)
            base_rng = dict(rng)
            cum_t = []
            ok = True
            for k, cs, an in cset:
                ups = [seq[i][1] for i in cs]
                los = [seq[i][1] for i in an][::-1]
                for l in ups + los:
                    base_rng[l] &= A
                    ok = ok and bool(base_rng[l])
                cum_t.append(("l%d" % k, tuple(ups + los)))
            if not ok:
                continue
            choices = []
            for i, j in pairs:
                li, lj = seq[i][1], seq[j][1]
                r = base_rng[li] & base_rng[lj]
                choices.append(_gamma_options(r) if seq[i][0] == UP else _eta_options(r))
            for pick in itertools.product(*choices):
                r2 = dict(base_rng)
                coef = x.coef * y.coef * sign
                tens = list(x.tensors) + list(y.tensors) + cum_t
                merge = {}
                for (i, j), (c, kind, rr) in zip(pairs, pick):
                    li, lj = seq[i][1], seq[j][1]
                    coef *= c
                    r2[li] &= rr
                    r2[lj] &= rr
                    if kind == "delta":
                        merge[lj] = li
                    elif seq[i][0] == UP:            # gamma-type: rows = creator label
                        tens.append((kind, (li, lj)))
                    else:                            # eta-type: rows = creator label (right string)
                        tens.append((kind, (lj, li)))
                if merge:
                    tens = [(nm, tuple(merge.get(l, l) for l in ls)) for nm, ls in tens]
                    for l in merge:
                        del r2[l]
                up = [seq[i][1] for i in free_up]
                lo = [seq[i][1] for i in free_lo][::-1]
                out.append(SOTerm(coef, tens, up, lo, r2,
                                  x.has_l2 or y.has_l2 or any(k == 2 for k, _, _ in cset)))
    return out


def _matchings(seq, rng, xs, ys):
    res = []

    def go(a, used, acc):
        if a == len(xs):
            res.append(list(acc))
            return
        go(a + 1, used, acc)
        i = xs[a]
        for j in ys:
            if j in used or seq[i][0] == seq[j][0]:
                continue
            r = rng[seq[i][1]] & rng[seq[j][1]]
            ok = (r & H) if seq[i][0] == UP else (r & P)
            if ok:
                acc.append((i, j))
                go(a + 1, used | {j}, acc)
                acc.pop()

    go(0, frozenset(), [])
    return res


def _fresh(term: SOTerm, start):
    m = {}
    for l in sorted(term.labels()):
        m[l] = start + len(m)
    return SOTerm(term.coef, [(n, tuple(m[l] for l in ls)) for n, ls in term.tensors],
                  [m[l] for l in term.upper], [m[l] for l in term.lower],
                  {m[l]: r for l, r in term.rng.items()}, term.has_l2)


def commutator(xs, ys, max_rank=None):
    out = []
    for x in xs:
        for y in ys:
            xa = _fresh(x, 0)
            yb = _fresh(y, 1000)
            out += wick_product(xa, yb, max_rank)
            for t in wick_product(yb, xa, max_rank):
                t.coef = -t.coef
                out.append(t)
    return out


# ---- operators of the theory -------------------------------------------------------

def hamiltonian():
    f = SOTerm(Fraction(1), [("f", (0, 1))], [0], [1], {0: G, 1: G})
    v = SOTerm(Fraction(1, 4), [("v", (0, 1, 2, 3))], [0, 1], [2, 3], {i: G for i in range(4)})
    return [f, v]


def cluster(r1=(H, P), r2=(H, H, P, P)):
    """T1 + T2 with legs on the given ranges; t1(k,c) = t^c_k, t2(k,l,c,d) = t^{cd}_{kl}."""
    out = []
    if r1 is not None:
        out.append(SOTerm(Fraction(1), [("t1", (0, 1))], [1], [0], {0: r1[0], 1: r1[1]}))
    if r2 is not None:
        out.append(SOTerm(Fraction(1, 4), [("t2", (0, 1, 2, 3))], [2, 3], [0, 1],
                          {0: r2[0], 1: r2[1], 2: r2[2], 3: r2[3]}))
    return out


# ---- spin integration -----------------------------------------------------------------

def _s3():
    return list(itertools.permutations(range(3)))


def k3_weights():
    """Weights w_pi with K3[pqr;stu] = sum_pi w_pi Lambda3[pqr; pi(stu)].

    The loop-count element X = sum_pi sgn(pi) 2^cycles(pi) pi of the group algebra
    of S_3 acts as 0 on the trivial, 24 on the sign and 6 on the standard
    representation; its pseudo-inverse is (1/24) P_sign + (1/6) P_std.
    """
    w = {}
    for p in _s3():
        sgn = _sign_of(p)
        fixed = sum(1 for i in range(3) if p[i] == i)
        chi_std = {3: 2, 1: 0, 0: -1}[fixed]
        w[p] = Fraction(sgn, 24) / 6 + Fraction(1, 6) * Fraction(2, 6) * chi_std
    return w


def _structures(name, ls):
    """Spin structures of one spin-orbital factor: [(coef, (spatial name, labels), pairs)]."""
    if name in ("f", "gA", "eA"):
        return [(1, (name, ls), [(ls[0], ls[1])])]
    if name == "t1":
        k, c = ls
        return [(1, ("T1", (k, c)), [(c, k)])]
    if name == "v":
        p, q, r, s = ls
        return [(1, ("eri", (p, r, q, s)), [(p, r), (q, s)]),
                (-1, ("eri", (p, s, q, r)), [(p, s), (q, r)])]
    if name == "t2":
        k, l, c, d = ls
        return [(1, ("T2", (k, l, c, d)), [(c, k), (d, l)]),
                (-1, ("T2", (k, l, d, c)), [(c, l), (d, k)])]
    if name == "l2":
        p, q, r, s = ls
        return [(1, ("K2", (p, q, r, s)), [(p, r), (q, s)]),
                (-1, ("K2", (p, q, s, r)), [(p, s), (q, r)])]
    if name == "l3":
        up, lo = ls[:3], ls[3:]
        out = []
        for pi in _s3():
            low = tuple(lo[pi[i]] for i in range(3))
            out.append((_sign_of(pi), ("K3", tuple(up) + low), [(up[i], low[i]) for i in range(3)]))
        return out
    raise KeyError(name)


@dataclass
class SFTerm:
    """Spin-free term: coef * prod(factors), summed over internal labels, into out[ext labels]."""
    coef: Fraction
    factors: list            # [(name, labels)]
    ext: tuple               # output labels in output-axis order
    rng: dict


def spin_integrate(t: SOTerm, ext_labels, ext_spins):
    """Spin-free terms of one spin-orbital term with external labels at fixed spins (0=a,1=b)."""
    per = [_structures(n, ls) for n, ls in t.tensors]
    spin_of = dict(zip(ext_labels, ext_spins))
    out = []
    for pick in itertools.product(*per):
        coef = t.coef
        adj = {}
        facs = []
        for c, fac, pairs in pick:
            coef *= c
            facs.append(fac)
            for a, b in pairs:
                adj.setdefault(a, []).append(b)
                adj.setdefault(b, []).append(a)
        # walk components of the delta graph
        seen = set()
        loops = 0
        ok = True
        for start in adj:
            if start in seen:
                continue
            comp = []
            stack = [start]
            seen.add(start)
            while stack:
                u = stack.pop()
                comp.append(u)
                for w in adj[u]:
                    if w not in seen:
                        seen.add(w)
                        stack.append(w)
            ex = [u for u in comp if u in spin_of]
            if not ex:
                loops += 1
            else:
                if len({spin_of[u] for u in ex}) > 1:
                    ok = False
                    break
        if not ok:
            continue
        coef *= 2 ** loops
        if coef != 0:
            out.append(SFTerm(coef, facs, tuple(ext_labels), dict(t.rng)))
    return out


# ---- canonical form of spin-free terms ------------------------------------------------

# index symmetries of spatial tensors: list of label-position permutations that leave the value unchanged
SYMMETRIES = {
    "eri": [(0, 1, 2, 3), (1, 0, 2, 3), (0, 1, 3, 2), (1, 0, 3, 2),
            (2, 3, 0, 1), (3, 2, 0, 1), (2, 3, 1, 0), (3, 2, 1, 0)],
    "T2": [(0, 1, 2, 3), (1, 0, 3, 2)],
    "K2": [(0, 1, 2, 3), (1, 0, 3, 2), (2, 3, 0, 1), (3, 2, 1, 0)],
    "K3": None,   # filled below: simultaneous column permutations and upper<->lower
    "f": [(0, 1), (1, 0)],
    "gA": [(0, 1), (1, 0)],
    "eA": [(0, 1), (1, 0)],
}


def _k3_syms():
    out = []
    for pi in _s3():
        base = tuple(pi) + tuple(3 + pi[i] for i in range(3))
        out.append(base)
        out.append(tuple(base[3:]) + tuple(base[:3]))
    return out


SYMMETRIES["K3"] = _k3_syms()


def canonical_key(t: SFTerm):
    """A key equal for terms that are the same after renaming internal labels and
    using the index symmetries of the spatial tensors (greedy; equal keys are exact)."""
    ext_pos = {l: i for i, l in enumerate(t.ext)}
    best = None
    facs = t.factors
    # order factors by name/ranges, try the few orderings of identical-signature factors
    def sig(f):
        n, ls = f
        return (n, tuple(t.rng[l] for l in ls))
    groups = {}
    for f in facs:
        groups.setdefault(sig(f), []).append(f)
    keys = sorted(groups)
    orders = [[]]
    for k in keys:
        grp = groups[k]
        perms = list(itertools.permutations(grp)) if len(grp) <= 3 else [tuple(grp)]
        orders = [o + list(p) for o in orders for p in perms]
    for order in orders[:24]:
        names = {}
        rep = []
        for n, ls in order:
            syms = SYMMETRIES.get(n, [tuple(range(len(ls)))])
            cands = []
            for s in syms:
                lp = tuple(ls[i] for i in s)
                enc = []
                tmp = dict(names)
                for l in lp:
                    if l in ext_pos:
                        enc.append(("e", ext_pos[l], t.rng[l]))
                    else:
                        if l not in tmp:
                            tmp[l] = len(tmp)
                        enc.append(("i", tmp[l], t.rng[l]))
                cands.append((tuple(enc), lp))
            enc, lp = min(cands)
            for l in lp:
                if l not in ext_pos and l not in names:
                    names[l] = len(names)
            rep.append((n, enc))
        key = tuple(rep)
        if best is None or key < best:
            best = key
    return best


def merge_sf(terms):
    acc = {}
    rep = {}
    for t in terms:
        k = canonical_key(t)
        if k in acc:
            acc[k] += t.coef
        else:
            acc[k] = t.coef
            rep[k] = t
    out = []
    for k, c in acc.items():
        if c != 0:
            t = rep[k]
            out.append(SFTerm(c, t.factors, t.ext, t.rng))
    return out


def merge_pair_images(s2_terms):
    """Merge S2 terms modulo the pair swap (k,l,c,d) -> (l,k,d,c).

    Only S2 + S2^T(pairs) enters R2, so a term and the pair-swapped image of
    another are interchangeable: each term is replaced by whichever of itself and
    its image has the smaller canonical key, and equal keys are summed.
    """
    acc = {}
    rep = {}
    for t in s2_terms:
        k, l, c, d = t.ext
        img = SFTerm(t.coef, t.factors, (l, k, d, c), t.rng)
        key, kimg = canonical_key(t), canonical_key(img)
        if kimg < key:
            key, t = kimg, img
        acc[key] = acc.get(key, 0) + t.coef
        rep.setdefault(key, t)
    return [SFTerm(c, rep[k].factors, rep[k].ext, rep[k].rng) for k, c in acc.items() if c != 0]


# ---- the residual and energy equations ----------------------------------------------------

EXT_T2_RANGES = (C, C, V, V)
EXT_T1_RANGES = (C, V)
T3_BLOCKS = [(C, A, A, A), (A, C, A, A), (A, A, A, V), (A, A, V, A)]


def derive():
    """Spin-free terms of E_corr, R1[k,c] and S2[k,l,c,d] (R2 = S2 + S2 with both pairs swapped)."""
    e, groups = derive_groups()
    r1 = merge_sf(groups["lin"][0] + groups["quad"][0])
    s2 = merge_pair_images(merge_sf(groups["lin"][1] + groups["quad"][1]))
    return e, r1, s2


def derive_groups():
    """Spin-free terms of E_corr, and of R1 and S2 by term group: "lin" (H + [H,T]) and "quad"
    (the filtered two-fold commutator), each group merged on its own.

    Linear part: H + [H,T] in full.  Two-fold commutator (Section 2.2):
      residuals: 1/2 ([[H,Te],T] + [[H,T],Te] - [[H,Te],Te]) without two-body cumulants,
                 Te = amplitudes without active indices (core->virtual);
      energy:    1/2 ([[H,T],T] - sum over three-active blocks b,b' of [[H,T_b],T_b']).
    """
    Hs = hamiltonian()
    T = cluster()
    Te = cluster(EXT_T1_RANGES, EXT_T2_RANGES)
    X = commutator(Hs, T, max_rank=3)
    Xe = commutator(Hs, Te, max_rank=3)
    lin = Hs + [x for x in X if x.rank() <= 2]
    quadR = ([(Fraction(1, 2), q) for q in commutator(Xe, T, 2)]
             + [(Fraction(1, 2), q) for q in commutator(X, Te, 2)]
             + [(Fraction(-1, 2), q) for q in commutator(Xe, Te, 2)])
    quadR = [(c, q) for c, q in quadR if not q.has_l2 and q.rank() in (1, 2)]
    quadE = [(Fraction(1, 2), q) for q in commutator(X, T, 0)]
    for rb in T3_BLOCKS:
        Xb = commutator(Hs, cluster(None, rb), max_rank=3)
        for rb2 in T3_BLOCKS:
            quadE += [(Fraction(-1, 2), q) for q in commutator(Xb, cluster(None, rb2), 0)]

    e_terms = []
    r1_by = {"lin": [], "quad": []}
    s2_by = {"lin": [], "quad": []}
    items = ([(Fraction(1), t, "lin") for t in lin] + [(c, q, "quad") for c, q in quadR]
             + [(c, q, "quad") for c, q in quadE])
    for c, t, grp in items:
        r1_terms, s2_terms = r1_by[grp], s2_by[grp]
        t = SOTerm(t.coef * c, t.tensors, t.upper, t.lower, t.rng, t.has_l2)
        r = t.rank()
        if r == 0:
            e_terms += spin_integrate(t, (), ())
        elif r == 1:
            u, l = t.upper[0], t.lower[0]
            rr = dict(t.rng)
            rr[u] &= P
            rr[l] &= H
            if not rr[u] or not rr[l]:
                continue
            t2 = SOTerm(t.coef, t.tensors, t.upper, t.lower, rr, t.has_l2)
            r1_terms += spin_integrate(t2, (l, u), (0, 0))          # R1[k, c]
        elif r == 2:
            u1, u2 = t.upper
            l1, l2 = t.lower
            rr = dict(t.rng)
            for x in (u1, u2):
                rr[x] &= P
            for x in (l1, l2):
                rr[x] &= H
            if not all(rr[x] for x in (u1, u2, l1, l2)):
                continue
            t2 = SOTerm(t.coef, t.tensors, t.upper, t.lower, rr, t.has_l2)
            # eq. (antisym) restricted to the alpha-beta sector; the pair-swapped half is
            # restored by the final symmetrization R2 = S2 + S2^T(pairs).
            s2_terms += spin_integrate(t2, (l1, l2, u1, u2), (0, 1, 0, 1))
            neg = SOTerm(-t.coef, t.tensors, t.upper, t.lower, rr, t.has_l2)
            s2_terms += spin_integrate(neg, (l1, l2, u2, u1), (0, 1, 0, 1))
    groups = {g: (merge_sf(r1_by[g]), merge_pair_images(merge_sf(s2_by[g]))) for g in ("lin", "quad")}
    return merge_sf(e_terms), groups
