"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Bar: fp64 residuals within 1e-10 relative (max |diff| / max |oracle|; where the oracle's
array is exactly zero, the difference itself), energies within 1e-9 E_h; integer/structural
properties exact.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

RTOL = 1e-10
ETOL = 1e-9


def _ctx(cfg, inp):
    from paper_2511_03567_amd import ric
    dev = torch.device("cuda", 0)
    ctx = ric.Context(0)
    ctx.set_spaces(cfg.nc, cfg.na, cfg.nv, cfg.naux)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx.load_fock(t(inp.f))
    ctx.load_df(t(inp.B))
    if cfg.na:
        ctx.load_rdms(t(inp.G1), t(inp.G2), t(inp.G3))
    else:
        ctx.load_rdms(None, None, None)
    return ctx, t


def _amps(cfg, seed, scale=0.05):
    rng = np.random.default_rng(seed)
    nH, nP = cfg.nc + cfg.na, cfg.na + cfg.nv
    m1, m2 = R.block_mask(cfg.nc, cfg.na, cfg.nv)
    T1 = rng.standard_normal((nH, nP)) * scale * m1
    T2 = rng.standard_normal((nH, nH, nP, nP)) * scale
    T2 = 0.5 * (T2 + T2.transpose(1, 0, 3, 2)) * m2
    return T1, T2


def _rel(a, b):
    """max |a - b| / max |b|; the plain difference where b is exactly zero."""
    if b.size == 0:
        return 0.0
    scale = float(np.abs(b).max())
    d = float(np.abs(a - b).max())
    return d / scale if scale > 0.0 else d


CASES = [
    ("tiny CAS(4,4) nc2 nv10 naux48", S.CONFIGS["tiny_cas44"]),
    ("CAS(4,4) nc3 nv20 naux30", S.custom_config("c3", 3, 4, 20, 30, 7)),
    ("single reference nc4 nv9 naux20", S.custom_config("sr", 4, 0, 9, 20, 8)),
    ("no core CAS(2,2) nv7 naux15", S.custom_config("nocore", 0, 2, 7, 15, 9)),
    ("CAS(6,6) nc2 nv11 naux25", S.custom_config("cas66", 2, 6, 11, 25, 10)),
    ("no virtuals nc3 CAS(3,3) naux10", S.custom_config("nov", 3, 3, 0, 10, 14)),
    ("active space only CAS(4,4) naux9", S.custom_config("cas", 0, 4, 0, 9, 15)),
    ("one of each nc1 na1 nv1 naux3", S.custom_config("one", 1, 1, 1, 3, 16)),
    ("single active orbital nc2 na1 nv3 naux5", S.custom_config("na1", 2, 1, 3, 5, 17)),
]


@pytest.mark.parametrize("name,cfg", CASES, ids=[c[0] for c in CASES])
def test_residual_energy_match_oracle(name, cfg):
    print(f"case {name}", flush=True)
    inp = S.make_inputs(cfg)
    ctx, t = _ctx(cfg, inp)
    T1, T2 = _amps(cfg, 3)
    nH, nP = cfg.nc + cfg.na, cfg.na + cfg.nv
    R1 = torch.full((nH, nP), 7.0, dtype=torch.float64, device="cuda")
    R2 = torch.full((nH, nH, nP, nP), 7.0, dtype=torch.float64, device="cuda")
    ctx.residual(t(T1), t(T2), R1, R2)
    e, e0 = ctx.energy(t(T1), t(T2))
    ref = R.Reference(cfg.nc, cfg.na, cfg.nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
    r1, r2 = ref.residual(T1, T2)
    assert _rel(R1.cpu().numpy(), r1) < RTOL
    assert _rel(R2.cpu().numpy(), r2) < RTOL
    assert abs(e - ref.energy(T1, T2)) < ETOL
    assert abs(e0 - ref.reference_energy()) < ETOL
    # the excluded all-active blocks are exactly zero; pair symmetry holds exactly
    g2 = R2.cpu().numpy()
    assert np.all(g2[cfg.nc:, cfg.nc:, :cfg.na, :cfg.na] == 0.0)
    assert np.array_equal(g2, g2.transpose(1, 0, 3, 2))


@pytest.mark.slow
def test_residual_matches_oracle_multi_tile():
    """nH*nP = 640 rows: ring contractions span several 128-wide tiles with a ragged tail."""
    cfg = S.custom_config("mt", 6, 4, 60, 80, 11)
    inp = S.make_inputs(cfg)
    ctx, t = _ctx(cfg, inp)
    T1, T2 = _amps(cfg, 4, 0.03)
    nH, nP = cfg.nc + cfg.na, cfg.na + cfg.nv
    R1 = torch.zeros((nH, nP), dtype=torch.float64, device="cuda")
    R2 = torch.zeros((nH, nH, nP, nP), dtype=torch.float64, device="cuda")
    ctx.residual(t(T1), t(T2), R1, R2)
    ref = R.Reference(cfg.nc, cfg.na, cfg.nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
    r1, r2 = ref.residual(T1, T2)
    assert _rel(R1.cpu().numpy(), r1) < RTOL
    assert _rel(R2.cpu().numpy(), r2) < RTOL


def test_update_matches_oracle():
    cfg = S.custom_config("upd", 3, 4, 20, 30, 12)
    inp = S.make_inputs(cfg)
    ctx, t = _ctx(cfg, inp)
    T1, T2 = _amps(cfg, 5)
    rng = np.random.default_rng(6)
    m1, m2 = R.block_mask(cfg.nc, cfg.na, cfg.nv)
    r1 = rng.standard_normal(T1.shape) * m1
    r2 = rng.standard_normal(T2.shape)
    r2 = 0.5 * (r2 + r2.transpose(1, 0, 3, 2)) * m2
    gT1, gT2 = t(T1), t(T2)
    n2 = ctx.update(gT1, gT2, t(r1), t(r2), 0.5)
    D1, D2 = R.denominators(inp.f, cfg.nc, cfg.na, cfg.nv)
    N1 = R.ric_update(T1, r1, D1, 0.5) * m1
    N2 = R.ric_update(T2, r2, D2, 0.5) * m2
    assert _rel(gT1.cpu().numpy(), N1) < 1e-14
    assert _rel(gT2.cpu().numpy(), N2) < 1e-14
    want = float(np.sum((N1 - T1) ** 2) + np.sum((N2 - T2) ** 2))
    assert abs(n2 - want) <= 1e-12 * want


def _ladder_sample(B, tau, nc, idx):
    """(ce|df) tau[k,l,e,f] for sampled (k,l,c,d), one element at a time."""
    Bp = B[:, nc:, nc:]
    out = []
    for k, l, c, d in idx:
        v = np.einsum("xe,xf,ef->", Bp[:, c, :], Bp[:, d, :], tau[k, l], optimize=True)
        out.append(v)
    return np.array(out)


@pytest.mark.parametrize("nc,na,nv,naux", [(5, 8, 193, 150), (1, 2, 3, 7)])
def test_ladder_matches_sampled_definition(nc, na, nv, naux):
    """R2 += sum_ef (ce|df) tau[k,l,e,f], nP = 201: several W and tau tiles with ragged tails."""
    print(f"ladder nc={nc} na={na} nv={nv} naux={naux}", flush=True)
    cfg = S.custom_config("lad", nc, na, nv, naux, 13, ci_fraction=1.0)
    rng = np.random.default_rng(13)
    n = nc + na + nv
    f = np.diag(np.arange(n, dtype=float))
    B = S.make_df(rng, n, naux)
    from paper_2511_03567_amd import ric
    ctx = ric.Context(0)
    ctx.set_spaces(nc, na, nv, naux)
    dev = torch.device("cuda", 0)
    ctx.load_fock(torch.from_numpy(f).to(dev))
    ctx.load_df(torch.from_numpy(B).to(dev))
    nH, nP = nc + na, na + nv
    tau = rng.standard_normal((nH, nH, nP, nP))
    tau = tau + tau.transpose(1, 0, 3, 2)
    R2 = torch.zeros((nH, nH, nP, nP), dtype=torch.float64, device=dev)
    ctx.ladder(torch.from_numpy(tau).to(dev), R2)
    got = R2.cpu().numpy()
    idx = [tuple(int(x) for x in (rng.integers(nH), rng.integers(nH), rng.integers(nP), rng.integers(nP)))
           for _ in range(64)]
    idx += [(0, 0, 0, 0), (nH - 1, nH - 1, nP - 1, nP - 1), (0, nH - 1, nP - 1, 0)]
    want = _ladder_sample(B, tau, nc, idx)
    g = np.array([got[i] for i in idx])
    assert np.abs(g - want).max() / np.abs(want).max() < RTOL
    assert np.array_equal(got, got.transpose(1, 0, 3, 2))


@pytest.mark.parametrize("precision", ["fp64", "fp32mix"])
def test_residual_with_padded_operands(monkeypatch, precision):
    """Every product with a K that is not a multiple of the load width gathered with zero padding
    (the path large products take), odd extents throughout: still the oracle's residual."""
    from paper_2511_03567_amd import ric
    monkeypatch.setenv("RIC_PAD_MIN_FLOPS", "0")
    monkeypatch.setenv("RIC_FP32_MIN_FLOPS", "0")   # mixed: every product with fp32 operands
    cfg = S.custom_config("odd", 3, 4, 21, 29, 18)
    inp = S.make_inputs(cfg)
    ctx, t = _ctx(cfg, inp)
    T1, T2 = _amps(cfg, 19)
    nH, nP = cfg.nc + cfg.na, cfg.na + cfg.nv
    R1 = torch.zeros((nH, nP), dtype=torch.float64, device="cuda")
    R2 = torch.zeros((nH, nH, nP, nP), dtype=torch.float64, device="cuda")
    prec = ric.RIC_FP64 if precision == "fp64" else ric.RIC_FP32MIX
    ctx.residual(t(T1), t(T2), R1, R2, prec)
    ref = R.Reference(cfg.nc, cfg.na, cfg.nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
    r1, r2 = ref.residual(T1, T2)
    tol = RTOL if precision == "fp64" else 1e-5
    assert _rel(R1.cpu().numpy(), r1) < tol
    assert _rel(R2.cpu().numpy(), r2) < tol


@pytest.mark.parametrize("name,cfg", [CASES[0], CASES[1], CASES[2], CASES[3]], ids=[c[0] for c in CASES[:4]])
def test_fock_from_core_hamiltonian(name, cfg):
    """f(h) on the GPU inverts the oracle's h(f) (generalized Fock matrix, Section 2.1)."""
    inp = S.make_inputs(cfg)
    ctx, t = _ctx(cfg, inp)
    ref = R.Reference(cfg.nc, cfg.na, cfg.nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
    h = ref.core_hamiltonian()
    f = torch.zeros((cfg.n, cfg.n), dtype=torch.float64, device="cuda")
    ctx.build_fock(t(h), f)
    assert _rel(f.cpu().numpy(), inp.f) < 1e-12


@pytest.mark.parametrize("name,cfg", [CASES[1], CASES[3], ("single reference nc4 nv9 naux20", CASES[2][1])],
                         ids=["cas44", "nocore", "sr"])
def test_semicanonical_rotation_is_covariant(name, cfg):
    """After semicanonicalization (block-diagonal orthogonal U), the residual at the rotated
    amplitudes is the rotated residual and the energy is unchanged (block-rotation covariance
    of the residual and energy functions); f' is diagonal within the core, active and virtual
    blocks and equals U^T f U."""
    print(f"semicanonical {name}", flush=True)
    inp = S.make_inputs(cfg)
    nc, na, nv = cfg.nc, cfg.na, cfg.nv
    nH, nP, n = nc + na, na + nv, cfg.n
    T1, T2 = _amps(cfg, 31)
    ctx, t = _ctx(cfg, inp)
    R1 = torch.zeros((nH, nP), dtype=torch.float64, device="cuda")
    R2 = torch.zeros((nH, nH, nP, nP), dtype=torch.float64, device="cuda")
    ctx.residual(t(T1), t(T2), R1, R2)
    e, _ = ctx.energy(t(T1), t(T2))
    U, fr = ctx.semicanonicalize()
    U, fr = U.cpu().numpy(), fr.cpu().numpy()
    assert np.abs(U.T @ U - np.eye(n)).max() < 1e-12
    assert np.abs(fr - U.T @ inp.f @ U).max() < 1e-12 * np.abs(inp.f).max()
    for a, b in ((0, nc), (nc, nc + na), (nc + na, n)):
        blk = fr[a:b, a:b]
        assert np.abs(blk - np.diag(np.diag(blk))).max(initial=0.0) < 1e-10
        assert np.abs(U[a:b, :a]).max(initial=0.0) == 0.0 and np.abs(U[a:b, b:]).max(initial=0.0) == 0.0
    uh, up = U[:nH, :nH], U[nc:, nc:]
    rot1 = lambda x: uh.T @ x @ up
    rot2 = lambda x: np.einsum("kK,lL,cC,dD,klcd->KLCD", uh, uh, up, up, x, optimize=True)
    S1 = torch.zeros_like(R1)
    S2 = torch.zeros_like(R2)
    ctx.residual(t(rot1(T1)), t(rot2(T2)), S1, S2)
    e2, _ = ctx.energy(t(rot1(T1)), t(rot2(T2)))
    assert _rel(S1.cpu().numpy(), rot1(R1.cpu().numpy())) < 1e-10
    assert _rel(S2.cpu().numpy(), rot2(R2.cpu().numpy())) < 1e-10
    assert abs(e2 - e) < 1e-10


def test_triplet_reference_matches_oracle():
    """A triplet reference: spin-free RDMs of the M_S = 1 component (equal to those of M_S = 0),
    unchanged equations; the GPU residual and energy match the oracle."""
    nc, na, nv, naux = 2, 4, 12, 30
    cfg = S.custom_config("trip", nc, na, nv, naux, 47)
    inp = S.make_inputs(cfg, with_rdms=False)
    (d1, c1), (d0, c0) = S.random_triplet(np.random.default_rng(48), na)
    G = S.spinfree_rdms(d1, c1, na, 3)
    G0 = S.spinfree_rdms(d0, c0, na, 3)
    from paper_2511_03567_amd import ric
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    T1, T2 = _amps(cfg, 49)
    nH, nP = nc + na, na + nv
    out = []
    for GG in (G, G0):
        ctx = ric.Context(0)
        ctx.set_spaces(nc, na, nv, naux)
        ctx.load_fock(t(inp.f))
        ctx.load_df(t(inp.B))
        ctx.load_rdms(*(t(g) for g in GG))
        R1 = torch.zeros((nH, nP), dtype=torch.float64, device=dev)
        R2 = torch.zeros((nH, nH, nP, nP), dtype=torch.float64, device=dev)
        ctx.residual(t(T1), t(T2), R1, R2)
        e, _ = ctx.energy(t(T1), t(T2))
        out.append((R1.cpu().numpy(), R2.cpu().numpy(), e))
    ref = R.Reference(nc, na, nv, inp.f, inp.B, *G)
    r1, r2 = ref.residual(T1, T2)
    assert _rel(out[0][0], r1) < RTOL and _rel(out[0][1], r2) < RTOL
    assert abs(out[0][2] - ref.energy(T1, T2)) < ETOL
    assert _rel(out[1][1], out[0][1]) < 1e-12 and abs(out[1][2] - out[0][2]) < 1e-12


@pytest.mark.parametrize("name,cfg", [CASES[0], CASES[4], CASES[8]], ids=[CASES[i][0] for i in (0, 4, 8)])
def test_term_groups_match_oracle_groups(name, cfg):
    """ric_residual's term mask: the linear group H + [H,T] and the filtered two-fold commutator each
    match the oracle's group of the same name; the ladder and non-ladder parts of each group add up
    to the group, and the two groups to the residual."""
    from paper_2511_03567_amd import ric
    print(f"term groups {name}", flush=True)
    inp = S.make_inputs(cfg)
    ctx, t = _ctx(cfg, inp)
    T1, T2 = _amps(cfg, 41)
    nH, nP = cfg.nc + cfg.na, cfg.na + cfg.nv
    gT1, gT2 = t(T1), t(T2)
    ref = R.Reference(cfg.nc, cfg.na, cfg.nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)

    def res(mask):
        R1 = torch.full((nH, nP), 7.0, dtype=torch.float64, device="cuda")
        R2 = torch.full((nH, nH, nP, nP), 7.0, dtype=torch.float64, device="cuda")
        ctx.residual(gT1, gT2, R1, R2, ric.RIC_FP64, mask)
        return R1.cpu().numpy(), R2.cpu().numpy()

    full = res(ric.RIC_TERMS_ALL)
    parts = {}
    for grp, bit in (("lin", ric.RIC_TERMS_LINEAR), ("quad", ric.RIC_TERMS_QUADRATIC)):
        g = res(bit | ric.RIC_TERMS_LADDER | ric.RIC_TERMS_NONLADDER)
        want = ref.residual(T1, T2, groups=(grp,))
        assert _rel(g[0], want[0]) < RTOL and _rel(g[1], want[1]) < RTOL, grp
        lad = res(bit | ric.RIC_TERMS_LADDER)
        non = res(bit | ric.RIC_TERMS_NONLADDER)
        for a, b, c in zip(lad, non, g):
            assert np.abs(a + b - c).max() <= 1e-12 * np.abs(c).max()
        assert np.array_equal(lad[1], lad[1].transpose(1, 0, 3, 2))
        parts[grp] = g
    for i in range(2):
        assert np.abs(parts["lin"][i] + parts["quad"][i] - full[i]).max() <= 1e-12 * np.abs(full[i]).max()
    with pytest.raises(ric.RicError):
        res(ric.RIC_TERMS_LINEAR)          # no ladder / non-ladder part selected
    with pytest.raises(ric.RicError):
        res(16)


def test_layout_classes_tile_the_dense_arrays():
    """ric_layout: the 3 singles and 9 doubles classes of Section 3.2, their pair images and the
    excluded all-active blocks cover the dense T1 / T2 arrays exactly once.  IJAB, IJTU and TUAB
    (both holes and both particles in one space) are their own pair images; the other six are not."""
    cfg = S.custom_config("lay", 3, 4, 5, 9, 43)
    inp = S.make_inputs(cfg)
    ctx, _ = _ctx(cfg, inp)
    lay = ctx.layout()
    nc, na, nv = cfg.nc, cfg.na, cfg.nv
    nH, nP = nc + na, na + nv
    assert sorted(lay) == sorted(["IA", "IT", "TA", "IJAB", "IJTU", "TUAB", "ITAB", "ITUV", "IJTA", "TUVA",
                                  "ITUA1", "ITUA2"])
    c1 = np.zeros((nH, nP), dtype=int)
    c2 = np.zeros((nH, nH, nP, nP), dtype=int)
    for name, (rank, st, ex) in lay.items():
        sl = tuple(slice(a, a + b) for a, b in zip(st, ex))
        if rank == 1:
            c1[sl] += 1
        else:
            c2[sl] += 1
            own = (st[0], ex[0]) == (st[1], ex[1]) and (st[2], ex[2]) == (st[3], ex[3])
            assert own == (name in ("IJAB", "IJTU", "TUAB")), name
            if not own:                         # the pair image is a block of its own
                img = np.zeros_like(c2)
                img[sl] = 1
                c2 += img.transpose(1, 0, 3, 2)
    c1[nc:, :na] += 1                          # excluded: active -> active
    c2[nc:, nc:, :na, :na] += 1                # excluded: all four active
    assert np.all(c1 == 1) and np.all(c2 == 1)


def test_borrowed_df_factors_give_the_same_residual():
    """ric_load_df(borrow=1) uses the caller's B in place: same residual, energy and update as a copy."""
    from paper_2511_03567_amd import ric
    cfg = CASES[1][1]
    inp = S.make_inputs(cfg)
    T1, T2 = _amps(cfg, 45)
    out = []
    for borrow in (False, True):
        ctx, t = _ctx(cfg, inp)
        Bd = t(inp.B)
        ctx.load_df(Bd, borrow=borrow)
        nH, nP = cfg.nc + cfg.na, cfg.na + cfg.nv
        R1 = torch.zeros((nH, nP), dtype=torch.float64, device="cuda")
        R2 = torch.zeros((nH, nH, nP, nP), dtype=torch.float64, device="cuda")
        ctx.residual(t(T1), t(T2), R1, R2)
        e, _ = ctx.energy(t(T1), t(T2))
        out.append((R1.cpu().numpy(), R2.cpu().numpy(), e))
        ctx.close()
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][1], out[1][1])
    assert out[0][2] == out[1][2]


def _semicanonical_cpu(f, nc, na, nv):
    """Block eigenvectors of f (numpy), each column's entry of largest magnitude made positive."""
    n = nc + na + nv
    U = np.zeros((n, n))
    for a, b in ((0, nc), (nc, nc + na), (nc + na, n)):
        if b == a:
            continue
        _, v = np.linalg.eigh(f[a:b, a:b])
        piv = np.argmax(np.abs(v), axis=0)
        v = v * np.where(v[piv, np.arange(v.shape[1])] < 0, -1.0, 1.0)
        U[a:b, a:b] = v
    return U


@pytest.mark.parametrize("name,cfg", [CASES[1], CASES[3], CASES[2]], ids=["cas44", "nocore", "sr"])
def test_semicanonical_residual_matches_oracle_on_rotated_inputs(name, cfg):
    """After ric_semicanonicalize, the residual and energy at seeded amplitudes (in the new orbitals)
    equal the oracle's on f, B and the RDMs rotated by block eigenvectors computed with numpy under
    the same sign convention; U itself matches."""
    print(f"semicanonical vs oracle {name}", flush=True)
    inp = S.make_inputs(cfg)
    nc, na, nv = cfg.nc, cfg.na, cfg.nv
    nH, nP = nc + na, na + nv
    ctx, t = _ctx(cfg, inp)
    Ug, _ = ctx.semicanonicalize()
    U = _semicanonical_cpu(inp.f, nc, na, nv)
    assert np.abs(Ug.cpu().numpy() - U).max() < 1e-10
    fr = U.T @ inp.f @ U
    Br = np.einsum("pi,Xpq,qj->Xij", U, inp.B, U, optimize=True)
    ua = U[nc:nc + na, nc:nc + na]
    rot = lambda G: np.einsum(("ai,bj," if G.ndim == 2 else "ai,bj,ck,dl," if G.ndim == 4 else
                                "ai,bj,ck,dl,em,fn,") + "abcdef"[:G.ndim] + "->" + "ijklmn"[:G.ndim],
                               *([ua] * G.ndim), G, optimize=True)
    G1r, G2r, G3r = (rot(G) for G in (inp.G1, inp.G2, inp.G3)) if na else (inp.G1, inp.G2, inp.G3)
    T1, T2 = _amps(cfg, 47)
    R1 = torch.zeros((nH, nP), dtype=torch.float64, device="cuda")
    R2 = torch.zeros((nH, nH, nP, nP), dtype=torch.float64, device="cuda")
    ctx.residual(t(T1), t(T2), R1, R2)
    e, e0 = ctx.energy(t(T1), t(T2))
    ref = R.Reference(nc, na, nv, fr, Br, G1r, G2r, G3r)
    r1, r2 = ref.residual(T1, T2)
    assert _rel(R1.cpu().numpy(), r1) < RTOL and _rel(R2.cpu().numpy(), r2) < RTOL
    assert abs(e - ref.energy(T1, T2)) < ETOL
    assert abs(e0 - ref.reference_energy()) < ETOL
