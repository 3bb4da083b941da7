"""Full-size parity: the 809-orbital CAS(12,12) workload (nc=40, nv=757, naux=2200, the
benchmark's shapes and launch configuration) against the oracle on sampled outputs.

The amplitudes vanish outside a few cores and virtuals spread over the index ranges
(first and last orbitals, both sides of the 128-wide tile edge, the lone particle of the
ragged last tile, interior ones).  Every residual element whose indices lie in those
cores + all actives + those virtuals, and the correlation energy, then equal the
oracle's on the problem restricted to those orbitals; test_subset_cpu.py checks that
reduction with the oracle alone.  Bar: 1e-10 relative (max |diff| / max |oracle|) on the FP64 residuals, 1e-5 on
the FP32-mixed residuals (FP32 MFMA tiles, their partial sums added into FP64 every 128 terms of K), 1e-9 E_h on
the energy.  The regularized update, elementwise in the diagonal of f, is checked on the
same elements against the oracle's update of the oracle's own residual, to 1e-13 (the
residuals' rounding differences pass through the update's factor).

The adjoint (dT = J_r^T x) reduces the same way when x also vanishes outside the subset:
along amplitude directions inside the subset the full residual and the restricted one are
the same function.  Its subset part is checked by a dot-product test <x, J v> = <dT, v>
against central differences of the oracle on the subset, exact up to rounding because the
residual is quadratic in T.
"""
import time

import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R

import orbital_subset as OS

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

@pytest.fixture(autouse=True)
def _release_cached_memory():
    """The 809-orbital tests need most of the device, and the library allocates with hipMalloc:
    hand back to the driver what earlier tests left in torch's caching allocator (and contexts
    still awaiting collection) before each one."""
    import gc
    gc.collect()
    torch.cuda.empty_cache()
    yield


CORES = [0, 21, 38, 39]
VIRTS = [0, 115, 116, 390, 755, 756]     # particle positions 12, 127, 128, 402, 767, 768 of 769


@pytest.mark.timeout(900)
def test_fullsize_residual_and_energy_sampled():
    from paper_2511_03567_amd import ric
    cfg = S.CONFIGS["b12_cas1212"]
    nc, na, nv = cfg.nc, cfg.na, cfg.nv
    t0 = time.perf_counter()
    print(f"full size {cfg.name}: nc={nc} na={na} nv={nv} naux={cfg.naux}, cores {CORES}, virtuals {VIRTS}",
          flush=True)
    inp = S.make_inputs(cfg)
    fs, Bs = OS.restrict(inp.f, inp.B, nc, na, CORES, VIRTS)
    hm, pm = OS.hole_map(nc, na, CORES), OS.particle_map(na, VIRTS)
    ncs, nvs = len(CORES), len(VIRTS)
    rng = np.random.default_rng(11)
    m1, m2 = R.block_mask(ncs, na, nvs)
    T1s = rng.standard_normal((ncs + na, na + nvs)) * 0.05 * m1
    T2s = rng.standard_normal((ncs + na,) * 2 + (na + nvs,) * 2) * 0.05
    T2s = 0.5 * (T2s + T2s.transpose(1, 0, 3, 2)) * m2
    print(f"  inputs in {time.perf_counter() - t0:.1f} s", flush=True)

    dev = torch.device("cuda", 0)
    ctx = ric.Context(0)
    ctx.set_spaces(nc, na, nv, cfg.naux)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx.load_fock(t(inp.f))
    Bd = t(inp.B)
    ctx.load_df(Bd)
    del Bd
    ctx.load_rdms(t(inp.G1), t(inp.G2), t(inp.G3))
    G1, G2, G3 = inp.G1, inp.G2, inp.G3
    del inp
    s1, s2 = ctx.amplitude_shapes()
    h = torch.as_tensor(hm, device=dev)
    p = torch.as_tensor(pm, device=dev)
    i1 = (h[:, None], p[None, :])
    i2 = (h[:, None, None, None], h[None, :, None, None], p[None, None, :, None], p[None, None, None, :])
    T1 = torch.zeros(s1, dtype=torch.float64, device=dev)
    T2 = torch.zeros(s2, dtype=torch.float64, device=dev)
    T1[i1] = t(T1s)
    T2[i2] = t(T2s)
    R1 = torch.full(s1, 7.0, dtype=torch.float64, device=dev)
    R2 = torch.full(s2, 7.0, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    print("  energy at full size", flush=True)
    e, _ = ctx.energy(T1, T2)
    print("  FP32-mixed residual at full size", flush=True)
    ctx.residual(T1, T2, R1, R2, ric.RIC_FP32MIX)
    torch.cuda.synchronize()
    R1m = R1[i1].cpu().numpy()
    R2m = R2[i2].cpu().numpy()
    R1.fill_(7.0)
    R2.fill_(7.0)
    print("  FP64 residual at full size", flush=True)
    ctx.residual(T1, T2, R1, R2, ric.RIC_FP64)
    torch.cuda.synchronize()
    R1g = R1[i1].cpu().numpy()
    R2g = R2[i2].cpu().numpy()
    print("  regularized update at full size", flush=True)
    ctx.update(T1, T2, R1, R2, cfg.s)
    U1 = T1[i1].cpu().numpy()
    U2 = T2[i2].cpu().numpy()
    del R1, R2
    ctx.close()
    del T1, T2
    torch.cuda.empty_cache()
    print(f"  GPU done at {time.perf_counter() - t0:.1f} s; oracle on the {ncs}-core {nvs}-virtual subset",
          flush=True)

    sub = R.Reference(ncs, na, nvs, fs, Bs, G1, G2, G3)
    R1o, R2o = sub.residual(T1s, T2s)
    r1 = float(np.abs(R1g - R1o).max() / np.abs(R1o).max())
    r2 = float(np.abs(R2g - R2o).max() / np.abs(R2o).max())
    x1 = float(np.abs(R1m - R1o).max() / np.abs(R1o).max())
    x2 = float(np.abs(R2m - R2o).max() / np.abs(R2o).max())
    print(f"  residual rel diff FP64: R1 {r1:.2e} R2 {r2:.2e}; FP32-mixed: R1 {x1:.2e} R2 {x2:.2e}", flush=True)
    eo = sub.energy(T1s, T2s)
    print(f"  energy {e:.12f} oracle {eo:.12f} |dE| {abs(e - eo):.2e}; {time.perf_counter() - t0:.1f} s",
          flush=True)
    D1, D2 = R.denominators(fs, ncs, na, nvs)
    N1 = R.ric_update(T1s, R1o, D1, cfg.s) * m1
    N2 = R.ric_update(T2s, R2o, D2, cfg.s) * m2
    u1 = float(np.abs(U1 - N1).max() / np.abs(N1).max())
    u2 = float(np.abs(U2 - N2).max() / np.abs(N2).max())
    print(f"  update rel diff T1 {u1:.2e} T2 {u2:.2e}", flush=True)
    assert r1 < 1e-10 and r2 < 1e-10
    assert x1 < 1e-5 and x2 < 1e-5
    assert u1 < 1e-13 and u2 < 1e-13
    assert abs(e - eo) < 1e-9


CORES_ADJ = [0, 39]
VIRTS_ADJ = [115, 116, 756]
H = 1e-3


def _sym(rng, nh, np_, m2, scale):
    x = rng.standard_normal((nh, nh, np_, np_)) * scale
    return 0.5 * (x + x.transpose(1, 0, 3, 2)) * m2


@pytest.mark.timeout(900)
def test_fullsize_adjoint_residual_sampled():
    from paper_2511_03567_amd import ric
    cfg = S.CONFIGS["b12_cas1212"]
    nc, na, nv = cfg.nc, cfg.na, cfg.nv
    t0 = time.perf_counter()
    print(f"full-size adjoint {cfg.name}: cores {CORES_ADJ}, virtuals {VIRTS_ADJ}", flush=True)
    inp = S.make_inputs(cfg)
    fs, Bs = OS.restrict(inp.f, inp.B, nc, na, CORES_ADJ, VIRTS_ADJ)
    hm, pm = OS.hole_map(nc, na, CORES_ADJ), OS.particle_map(na, VIRTS_ADJ)
    ncs, nvs = len(CORES_ADJ), len(VIRTS_ADJ)
    nhs, nps = ncs + na, na + nvs
    rng = np.random.default_rng(12)
    m1, m2 = R.block_mask(ncs, na, nvs)
    T = (rng.standard_normal((nhs, nps)) * 0.05 * m1, _sym(rng, nhs, nps, m2, 0.05))
    x = (rng.standard_normal((nhs, nps)) * m1, _sym(rng, nhs, nps, m2, 1.0))
    v = (rng.standard_normal((nhs, nps)) * m1, _sym(rng, nhs, nps, m2, 1.0))

    dev = torch.device("cuda", 0)
    ctx = ric.Context(0)
    ctx.set_spaces(nc, na, nv, cfg.naux)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx.load_fock(t(inp.f))
    Bd = t(inp.B)
    ctx.load_df(Bd)
    del Bd
    ctx.load_rdms(t(inp.G1), t(inp.G2), t(inp.G3))
    G = (inp.G1, inp.G2, inp.G3)
    del inp
    s1, s2 = ctx.amplitude_shapes()
    h = torch.as_tensor(hm, device=dev)
    p = torch.as_tensor(pm, device=dev)
    i1 = (h[:, None], p[None, :])
    i2 = (h[:, None, None, None], h[None, :, None, None], p[None, None, :, None], p[None, None, None, :])

    def full(a1, a2):
        b1 = torch.zeros(s1, dtype=torch.float64, device=dev)
        b2 = torch.zeros(s2, dtype=torch.float64, device=dev)
        b1[i1] = t(a1)
        b2[i2] = t(a2)
        return b1, b2

    T1, T2 = full(*T)
    X1, X2 = full(*x)
    dT1 = torch.full(s1, 7.0, dtype=torch.float64, device=dev)
    dT2 = torch.full(s2, 7.0, dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    print(f"  inputs in {time.perf_counter() - t0:.1f} s; adjoint residual at full size", flush=True)
    ctx.adjoint_residual(T1, T2, X1, X2, dT1, dT2)
    torch.cuda.synchronize()
    d1 = dT1[i1].cpu().numpy()
    d2 = dT2[i2].cpu().numpy()
    sym = bool(torch.equal(dT2, dT2.permute(1, 0, 3, 2)))
    masked = bool(torch.all(dT2[nc:, nc:, :na, :na] == 0.0))
    ctx.close()
    del T1, T2, X1, X2, dT1, dT2
    torch.cuda.empty_cache()
    print(f"  GPU done at {time.perf_counter() - t0:.1f} s; oracle differences on the subset", flush=True)

    sub = R.Reference(ncs, na, nvs, fs, Bs, *G)
    rp = sub.residual(T[0] + H * v[0], T[1] + H * v[1])
    rm = sub.residual(T[0] - H * v[0], T[1] - H * v[1])
    want = float(sum(np.sum(a * (b - c)) for a, b, c in zip(x, rp, rm)) / (2 * H))
    got = float(np.sum(d1 * v[0]) + np.sum(d2 * v[1]))
    print(f"  <dT, v> {got:.12e}  <x, J v> {want:.12e}  rel {abs(got - want) / abs(want):.2e}; "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    assert abs(got - want) <= 1e-9 * abs(want)
    assert sym and masked
