"""Pins of the CPU oracle against quantities fixed by the paper and by exact algebra.

* spin-orbital RDMs rebuilt from spin-free ones by the singlet relations of
  Section 2.3.1 equal the RDMs of an S = 0 state computed directly;
  RDM partial traces; the three-body permutation sum rule (Section 2.3.1);
* E0 = <Psi0|H|Psi0> by brute force (Section 2.1, h recovered from f);
* the energy functional with the energy filter of Section 2.2 equals the
  brute-force <H + [H,T] + 1/2[[H,T],T]> - 1/2<[[H,T3],T3]> (T3: amplitudes with
  three active indices) for a multi-determinant singlet reference;
* the single-reference limit: many-body residuals equal projected residuals
  (Section 2.2), checked by brute force with an empty active space;
* closed forms: residual at T = 0 is (f_ck, (ck|dl)); linear energy at the
  first-order amplitudes is the MP2 energy;
* limits of the regularized update (eq. ric-update).
"""
import itertools

import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R
from tests.fockspace import Fock, GNO, Hamiltonian, embed_reference, spin_orbital_integrals


def _sym_pair(T2):
    return 0.5 * (T2 + T2.transpose(1, 0, 3, 2))


def _random_amplitudes(rng, nc, na, nv, scale=0.05):
    nH, nP = nc + na, na + nv
    m1, m2 = R.block_mask(nc, na, nv)
    T1 = rng.standard_normal((nH, nP)) * scale * m1
    T2 = _sym_pair(rng.standard_normal((nH, nH, nP, nP)) * scale) * m2
    return T1, T2


# ---------------------------------------------------------------------------------------
# RDMs and cumulants


@pytest.mark.parametrize("na", [2, 4])
def test_singlet_relations_rebuild_spinorbital_rdms(na):
    rng = np.random.default_rng(5)
    dets, c = S.project_singlet(rng, na)
    Gs = S.spinfree_rdms(dets, c, na, 3)
    gs = S.spinorbital_rdms(dets, c, na, 3)
    for k in range(3):
        rebuilt = R.spinorbital_tensor(Gs[k])
        assert np.abs(rebuilt - gs[k]).max() < 1e-12, k


def test_rdm_traces_and_sum_rule():
    rng = np.random.default_rng(6)
    na = 4
    dets, c = S.random_ci(rng, na)            # not a spin eigenstate
    G1, G2, G3 = S.spinfree_rdms(dets, c, na, 3)
    N = na
    assert abs(np.trace(G1) - N) < 1e-12
    assert np.abs(np.einsum("tuvu->tv", G2) - (N - 1) * G1).max() < 1e-12
    assert np.abs(np.einsum("tuxvwx->tuvw", G3) - (N - 2) * G2).max() < 1e-12
    perms = ["pqrstu", "prqstu", "qprstu", "rqpstu", "rpqstu", "qrpstu"]
    total = sum(np.einsum(p + "->pqrstu", G3) for p in perms)
    assert np.abs(total).max() < 1e-12


def test_spinfree_cumulant_formulas():
    """Spin sums of the spin-orbital cumulants equal the spin-free formulas (S = 0 state)."""
    rng = np.random.default_rng(7)
    na = 4
    dets, c = S.project_singlet(rng, na)
    G1, G2, G3 = S.spinfree_rdms(dets, c, na, 3)
    g1, g2, g3 = S.spinorbital_rdms(dets, c, na, 3)
    l2, l3 = R.spinorbital_cumulants(g1, g2, g3)

    def spin_sum(x):
        k = x.ndim // 2
        out = 0
        for sp in itertools.product((0, 1), repeat=k):
            idx = [np.arange(na) + s * na for s in sp] * 2
            out = out + x[np.ix_(*idx)]
        return out
    L2, L3 = R.spinfree_cumulants(G1, G2, G3)
    assert np.abs(spin_sum(l2) - L2).max() < 1e-12
    assert np.abs(spin_sum(l3) - L3).max() < 1e-12


# ---------------------------------------------------------------------------------------
# brute force in Fock space


class Brute:
    def __init__(self, nc, na, nv, naux, seed, singlet=True):
        rng = np.random.default_rng(seed)
        self.nc, self.na, self.nv = nc, na, nv
        n = self.n = nc + na + nv
        self.F = Fock(2 * n)
        if na:
            if singlet:
                dets, c = S.project_singlet(rng, na)
            else:
                dets, c = S.random_ci(rng, na)
        else:
            dets, c = np.array([0], dtype=np.uint64), np.array([1.0])
        self.psi = embed_reference(self.F, nc, na, n, dets, c)
        self.gno = GNO(self.F, self.psi)
        x = rng.standard_normal((n, n)) * 0.3
        h = np.diag(np.concatenate([rng.uniform(-3, -1, nc), rng.uniform(-0.5, 0.5, na),
                                    rng.uniform(1, 3, nv)])) + 0.5 * (x + x.T) * 0.2
        B = S.make_df(rng, n, naux)
        self.h, self.B = h, B
        h_so = np.zeros((2 * n, 2 * n))
        h_so[:n, :n] = h
        h_so[n:, n:] = h
        v_so = spin_orbital_integrals(B, n)
        self.H = Hamiltonian(self.F, h_so, v_so)
        # generalized Fock matrix (Section 2.1) with the exact spin-orbital 1-RDM of Psi0
        core = [s * n + i for s in (0, 1) for i in range(nc)]
        act = [s * n + nc + t for s in (0, 1) for t in range(na)]
        gam = np.array([[self.gno.rdm([p], [q]) for q in act] for p in act]) if na else np.zeros((0, 0))
        f_so = h_so + sum(v_so[:, m, :, m] for m in core)
        if na:
            f_so = f_so + np.einsum("ptqu,tu->pq", v_so[:, act][:, :, :, act], gam)
        self.f = f_so[:n, :n]
        if na:
            G1, G2, G3 = S.spinfree_rdms(dets, c, na, 3)
        else:
            G1, G2, G3 = np.zeros((0, 0)), np.zeros((0,) * 4), np.zeros((0,) * 6)
        self.ref = R.Reference(nc, na, nv, self.f, B, G1, G2, G3)

    def T_coeffs(self, T1, T2, keep=None):
        """Spin-orbital GNO coefficient tensors of T (optionally only some T2 blocks)."""
        sp = self.ref.sp
        n = self.n
        t1, t2 = R.spinorbital_amplitudes(sp, T1, T2)
        Hl, Pl = R._hole_so(sp), R._particle_so(sp)
        c1 = np.zeros((2 * n, 2 * n))
        c1[:, :] = t1.T                              # {a^c_k} coefficient at [c, k]
        c2 = np.zeros((2 * n,) * 4)
        blk = np.einsum("klcd->cdkl", t2) * 0.25
        c2[np.ix_(Pl, Pl, Hl, Hl)] = blk
        return {1: c1, 2: c2}

    def op(self, coeffs, vec, tag):
        return self.gno.operator_apply(coeffs, vec, tag)


def _expect_hbar_energy(b: Brute, Tc, T3c):
    psi = b.psi
    Hp = b.H.apply(psi)
    Tp = b.op(Tc, psi, "T.psi")
    HTp = b.H.apply(Tp)
    TTp = b.op(Tc, Tp, "T.Tpsi")
    THp = b.op(Tc, Hp, "T.Hpsi")
    THTp = b.op(Tc, HTp, "T.HTpsi")
    TTHp = b.op(Tc, THp, "T.THpsi")
    HTTp = b.H.apply(TTp)
    e = psi @ Hp + psi @ HTp - psi @ THp + 0.5 * (psi @ HTTp - 2 * psi @ THTp + psi @ TTHp)
    if T3c is not None:
        T3p = b.op(T3c, psi, "T3.psi")
        T3T3p = b.op(T3c, T3p, "T3.T3psi")
        HT3p = b.H.apply(T3p)
        T3Hp = b.op(T3c, Hp, "T3.Hpsi")
        T3HT3p = b.op(T3c, HT3p, "T3.HT3psi")
        T3T3Hp = b.op(T3c, T3Hp, "T3.T3Hpsi")
        HT3T3p = b.H.apply(T3T3p)
        e -= 0.5 * (psi @ HT3T3p - 2 * psi @ T3HT3p + psi @ T3T3Hp)
    return float(e)


@pytest.mark.slow
def test_reference_energy_bruteforce():
    b = Brute(1, 4, 1, 10, seed=21)
    e0 = float(b.psi @ b.H.apply(b.psi))
    assert abs(b.ref.reference_energy() - e0) < 1e-10


@pytest.mark.slow
def test_energy_functional_bruteforce():
    """E_CC of the filtered functional equals brute-force expectation values (multi-determinant)."""
    b = Brute(1, 4, 1, 10, seed=22)
    rng = np.random.default_rng(23)
    T1, T2 = _random_amplitudes(rng, 1, 4, 1, scale=0.1)
    nc, na = 1, 4
    # T3: the amplitudes with three active indices (ITUV and TUVA blocks)
    T3 = np.zeros_like(T2)
    T3[:nc, nc:, :na, :na] = T2[:nc, nc:, :na, :na]        # ITUV  (i,t | u,v)
    T3[nc:, :nc, :na, :na] = T2[nc:, :nc, :na, :na]
    T3[nc:, nc:, :na, na:] = T2[nc:, nc:, :na, na:]        # TUVA  (t,u | v,a)
    T3[nc:, nc:, na:, :na] = T2[nc:, nc:, na:, :na]
    Tc = b.T_coeffs(T1, T2)
    T3c = b.T_coeffs(np.zeros_like(T1), T3)
    T3c = {2: T3c[2]}
    want = _expect_hbar_energy(b, Tc, T3c)
    got = b.ref.reference_energy() + b.ref.energy(T1, T2)
    assert abs(got - want) < 1e-10, (got, want)


@pytest.mark.slow
def test_single_reference_limit_projected_residuals():
    """With no active orbitals, many-body residuals equal projected CC residuals (Section 2.2)."""
    nc, nv = 2, 3
    b = Brute(nc, 0, nv, 8, seed=31)
    rng = np.random.default_rng(32)
    T1, T2 = _random_amplitudes(rng, nc, 0, nv, scale=0.1)
    Tc = b.T_coeffs(T1, T2)
    psi, F, n = b.psi, b.F, b.n
    Hp = b.H.apply(psi)
    Tp = b.op(Tc, psi, "T.psi")
    HTp = b.H.apply(Tp)
    TTp = b.op(Tc, Tp, "T.Tpsi")
    THp = b.op(Tc, Hp, "T.Hpsi")
    THTp = b.op(Tc, HTp, "T.HTpsi")
    TTHp = b.op(Tc, THp, "T.THpsi")
    HTTp = b.H.apply(TTp)
    Hbar = Hp + HTp - THp + 0.5 * (HTTp - 2 * THTp + TTHp)
    R1, R2 = b.ref.residual(T1, T2)
    for i in range(nc):
        for a in range(nv):
            phi = F.string([nc + a], [i], psi)          # a^+_a a_i |Phi>, alpha spin
            assert abs(phi @ Hbar - R1[i, a]) < 1e-10
    for i, j in itertools.product(range(nc), repeat=2):
        for a, c in itertools.product(range(nv), repeat=2):
            phi = F.string([nc + a, n + nc + c], [i, n + j], psi)
            assert abs(phi @ Hbar - R2[i, j, a, c]) < 1e-10
    E = float(psi @ Hbar) - b.ref.reference_energy()
    assert abs(E - b.ref.energy(T1, T2)) < 1e-10


# ---------------------------------------------------------------------------------------
# closed forms and limits


def _small_ref(nc=2, na=2, nv=3, naux=12, seed=41):
    cfg = S.custom_config("pin", nc, na, nv, naux, seed)
    inp = S.make_inputs(cfg)
    return cfg, inp, R.Reference(nc, na, nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)


def test_residual_at_zero_amplitudes_is_hamiltonian():
    cfg, inp, ref = _small_ref()
    nc, na, nv = cfg.nc, cfg.na, cfg.nv
    nH, nP = nc + na, na + nv
    m1, m2 = R.block_mask(nc, na, nv)
    R1, R2 = ref.residual(np.zeros((nH, nP)), np.zeros((nH, nH, nP, nP)))
    assert np.abs(R1 - inp.f[:nH, nc:] * m1).max() < 1e-14
    eri = np.einsum("Xpq,Xrs->pqrs", inp.B, inp.B)
    assert np.abs(R2 - np.einsum("ckdl->klcd", eri[nc:, :nH, nc:, :nH]) * m2).max() < 1e-14
    assert ref.energy(np.zeros((nH, nP)), np.zeros((nH, nH, nP, nP))) == 0.0


def test_mp2_closed_form():
    """No active space, s -> infinity: the first step gives first-order amplitudes; the linear
    energy at them is E_MP2 = sum (ia|jb)[2(ia|jb) - (ib|ja)] / Delta."""
    nc, nv = 3, 5
    cfg, inp, ref = _small_ref(nc, 0, nv, 15, 42)
    f = np.diag(np.diag(inp.f))
    ref = R.Reference(nc, 0, nv, f, inp.B, inp.G1, inp.G2, inp.G3)
    D1, D2 = R.denominators(f, nc, 0, nv)
    R1, R2 = ref.residual(np.zeros((nc, nv)), np.zeros((nc, nc, nv, nv)))
    T2 = R.ric_update(np.zeros_like(R2), R2, D2, 1e12)
    T1 = R.ric_update(np.zeros_like(R1), R1, D1, 1e12)
    eri = np.einsum("Xpq,Xrs->pqrs", inp.B, inp.B)
    ov = eri[:nc, nc:, :nc, nc:]
    emp2 = float(np.einsum("iajb,ijab->", 2 * ov - ov.transpose(0, 3, 2, 1), T2))
    e_lin = ref.energy(T1, T2, groups=("lin",))
    assert abs(e_lin - emp2) < 1e-12
    direct = sum(ov[i, a, j, b] * (2 * ov[i, a, j, b] - ov[i, b, j, a]) / D2[i, j, a, b]
                 for i in range(nc) for j in range(nc) for a in range(nv) for b in range(nv))
    assert abs(e_lin - direct) < 1e-12


def test_regularized_update_limits():
    rng = np.random.default_rng(3)
    T = rng.standard_normal(50)
    Rr = rng.standard_normal(50)
    D = rng.uniform(-3, 3, 50)
    # s -> infinity: eq. cc-update, t + r / Delta
    assert np.allclose(R.ric_update(T, Rr, D, 1e8), T + Rr / D, rtol=1e-12)
    # s -> 0: amplitudes vanish
    assert np.abs(R.ric_update(T, Rr, D, 1e-14)).max() < 1e-12
    # Delta -> 0: bounded, (1 - exp(-s D^2)) / D ~ s D
    tiny = np.array([1e-9, -1e-12, 0.0])
    phi = R.regularizer(tiny, 0.5)
    assert np.allclose(phi, 0.5 * tiny, rtol=1e-9, atol=0)
    assert np.all(np.abs(R.ric_update(np.ones(3), np.ones(3), tiny, 0.5)) < 1e-8)


def test_pair_symmetry_of_residual():
    cfg, inp, ref = _small_ref()
    rng = np.random.default_rng(9)
    T1, T2 = _random_amplitudes(rng, cfg.nc, cfg.na, cfg.nv)
    R1, R2 = ref.residual(T1, T2)
    assert np.abs(R2 - R2.transpose(1, 0, 3, 2)).max() < 1e-13


def test_quadratic_polynomial_structure():
    """r is at most quadratic in T: r(2T) - 2 r(T) + r(0) = 2 r_quad(T)."""
    cfg, inp, ref = _small_ref()
    rng = np.random.default_rng(10)
    T1, T2 = _random_amplitudes(rng, cfg.nc, cfg.na, cfg.nv)
    z1, z2 = np.zeros_like(T1), np.zeros_like(T2)
    a = ref.residual(2 * T1, 2 * T2)
    b = ref.residual(T1, T2)
    c = ref.residual(z1, z2)
    q = ref.residual(T1, T2, groups=("quad",))
    for k in range(2):
        assert np.abs(a[k] - 2 * b[k] + c[k] - 2 * q[k]).max() < 1e-12
