"""The CAS(8,8) (nc=10, nv=120, naux=360) and CAS(14,14) (nc=20, nv=300, naux=900, sparse 1 % CAS
vector) workloads on the GPU.

1. Sampled parity against the oracle: amplitudes that vanish outside a few core and virtual
   orbitals (first and last ones, both sides of a 128-wide tile edge), so every residual element
   on (those cores + all actives + those virtuals) and the correlation energy equal the oracle's
   on the problem restricted to those orbitals (tests/test_subset_cpu.py checks the reduction).
   FP64 residual within 1e-10 relative (max |diff| / max |oracle|), energy within 1e-9 E_h, the
   regularized update against the oracle's update of its own residual within 1e-13; the
   FP32-mixed residual within 1e-5.
2. FP32-mixed against FP64 at dense amplitudes (std 1e-2 on every stored amplitude, as in the
   benchmark): max |R_mixed - R_fp64| / max |R_fp64| within 1e-5, the value printed.
"""
import time

import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R

import orbital_subset as OS

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

CASES = [("mixed_cas88", [0, 4, 9], [0, 63, 64, 119]),
         ("large_cas1414", [0, 11, 19], [0, 115, 116, 299])]


def _rel(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.timeout(600)
@pytest.mark.parametrize("name,cores,virts", CASES, ids=[c[0] for c in CASES])
def test_config_sampled_parity_and_dense_mixed(name, cores, virts):
    from paper_2511_03567_amd import ric
    cfg = S.CONFIGS[name]
    nc, na, nv = cfg.nc, cfg.na, cfg.nv
    t0 = time.perf_counter()
    print(f"{name}: nc={nc} na={na} nv={nv} naux={cfg.naux}, cores {cores}, virtuals {virts}", flush=True)
    inp = S.make_inputs(cfg)
    print(f"  inputs in {time.perf_counter() - t0:.1f} s", flush=True)
    fs, Bs = OS.restrict(inp.f, inp.B, nc, na, cores, virts)
    hm, pm = OS.hole_map(nc, na, cores), OS.particle_map(na, virts)
    ncs, nvs = len(cores), len(virts)
    rng = np.random.default_rng(21)
    m1, m2 = R.block_mask(ncs, na, nvs)
    T1s = rng.standard_normal((ncs + na, na + nvs)) * 0.05 * m1
    T2s = rng.standard_normal((ncs + na,) * 2 + (na + nvs,) * 2) * 0.05
    T2s = 0.5 * (T2s + T2s.transpose(1, 0, 3, 2)) * m2

    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = ric.Context(0)
    ctx.set_spaces(nc, na, nv, cfg.naux)
    ctx.load_fock(t(inp.f))
    ctx.load_df(t(inp.B))
    ctx.load_rdms(t(inp.G1), t(inp.G2), t(inp.G3))
    s1, s2 = ctx.amplitude_shapes()
    T1f, T2f = OS.embed(T1s, T2s, hm, pm, nc + na, na + nv)
    T1, T2 = t(T1f), t(T2f)
    R1 = torch.full(s1, 7.0, dtype=torch.float64, device=dev)
    R2 = torch.full(s2, 7.0, dtype=torch.float64, device=dev)
    ctx.residual(T1, T2, R1, R2, ric.RIC_FP32MIX)
    i1, i2 = np.ix_(hm, pm), np.ix_(hm, hm, pm, pm)
    R1m, R2m = R1.cpu().numpy()[i1], R2.cpu().numpy()[i2]
    ctx.residual(T1, T2, R1, R2, ric.RIC_FP64)
    R1g, R2g = R1.cpu().numpy()[i1], R2.cpu().numpy()[i2]
    e, _ = ctx.energy(T1, T2)
    ctx.update(T1, T2, R1, R2, cfg.s)
    U1, U2 = T1.cpu().numpy()[i1], T2.cpu().numpy()[i2]

    # dense amplitudes: FP32-mixed against FP64
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg.seed)
    D1 = torch.randn(s1, dtype=torch.float64, device=dev, generator=gen) * 1e-2
    D2 = torch.randn(s2, dtype=torch.float64, device=dev, generator=gen) * 1e-2
    D2 = 0.5 * (D2 + D2.permute(1, 0, 3, 2))
    D1[nc:, :na] = 0.0
    D2[nc:, nc:, :na, :na] = 0.0
    D2 = D2.contiguous()
    ctx.residual(D1, D2, R1, R2, ric.RIC_FP64)
    F1, F2 = R1.clone(), R2.clone()
    ctx.residual(D1, D2, R1, R2, ric.RIC_FP32MIX)
    dense = max((R1 - F1).abs().max().item(), (R2 - F2).abs().max().item()) / \
        max(F1.abs().max().item(), F2.abs().max().item())
    ctx.close()
    del R1, R2, F1, F2, D1, D2, T1, T2
    torch.cuda.empty_cache()
    print(f"  GPU done at {time.perf_counter() - t0:.1f} s; dense amplitudes: FP32-mixed vs FP64 "
          f"max |diff| / max |R| = {dense:.2e}; oracle on the {ncs}-core {nvs}-virtual subset", flush=True)

    sub = R.Reference(ncs, na, nvs, fs, Bs, inp.G1, inp.G2, inp.G3)
    R1o, R2o = sub.residual(T1s, T2s)
    eo = sub.energy(T1s, T2s)
    r = max(_rel(R1g, R1o), _rel(R2g, R2o))
    x = max(_rel(R1m, R1o), _rel(R2m, R2o))
    Dd1, Dd2 = R.denominators(fs, ncs, na, nvs)
    u = max(_rel(U1, R.ric_update(T1s, R1o, Dd1, cfg.s) * m1), _rel(U2, R.ric_update(T2s, R2o, Dd2, cfg.s) * m2))
    print(f"  residual rel diff FP64 {r:.2e}, FP32-mixed {x:.2e}; energy {e:.12f} oracle {eo:.12f} "
          f"|dE| {abs(e - eo):.2e}; update {u:.2e}; {time.perf_counter() - t0:.1f} s", flush=True)
    assert r < 1e-10
    assert x < 1e-5
    assert abs(e - eo) < 1e-9
    assert u < 1e-13
    assert dense < 1e-5
