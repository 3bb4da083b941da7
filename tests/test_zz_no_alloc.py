"""The allocation-free update (ric_update_noalloc) against ric_update, through the C ABI.

Both run the same kernels, so the updated amplitudes and the step norm must agree bit for
bit; both are also checked against the oracle's update (eq. ric-update) to 1e-14.  Two calls
in a row on one GPU, the second on a smaller problem, so the shared device array is reused
with a smaller input; the free device memory does not change across a call.
"""
import numpy as np
import pytest

import synthetic as S
from oracle import ricmrcc as R

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _case(nc, na, nv, naux, seed):
    from paper_2511_03567_amd import ric
    cfg = S.custom_config("noalloc", nc, na, nv, naux, seed)
    inp = S.make_inputs(cfg)
    dev = torch.device("cuda", 0)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx = ric.Context(0)
    ctx.set_spaces(nc, na, nv, naux)
    ctx.load_fock(t(inp.f))
    ctx.load_df(t(inp.B))
    ctx.load_rdms(t(inp.G1), t(inp.G2), t(inp.G3))
    rng = np.random.default_rng(seed + 100)
    m1, m2 = R.block_mask(nc, na, nv)
    nH, nP = nc + na, na + nv
    T1 = rng.standard_normal((nH, nP)) * 0.05 * m1
    T2 = rng.standard_normal((nH, nH, nP, nP)) * 0.05
    T2 = 0.5 * (T2 + T2.transpose(1, 0, 3, 2)) * m2
    r1 = rng.standard_normal((nH, nP)) * m1
    r2 = rng.standard_normal((nH, nH, nP, nP))
    r2 = 0.5 * (r2 + r2.transpose(1, 0, 3, 2)) * m2
    return cfg, inp, ctx, t, (T1, T2), (r1, r2)


def test_update_noalloc_matches_update_on_two_calls():
    s = 0.5
    for shape in ((3, 4, 20, 30, 51), (2, 2, 7, 10, 52)):   # the second call on a smaller problem
        print(f"allocation-free update nc,na,nv,naux = {shape[:4]}", flush=True)
        cfg, inp, ctx, t, (T1, T2), (r1, r2) = _case(*shape)
        a1, a2 = t(T1), t(T2)
        b1, b2 = t(T1), t(T2)
        g1, g2 = t(r1), t(r2)
        na2 = ctx.update(a1, a2, g1, g2, s)
        torch.cuda.synchronize()
        free0, _ = torch.cuda.mem_get_info()
        nb2 = ctx.update_noalloc(b1, b2, g1, g2, s)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert free1 == free0
        assert torch.equal(a1, b1) and torch.equal(a2, b2)
        assert na2 == nb2
        D1, D2 = R.denominators(inp.f, cfg.nc, cfg.na, cfg.nv)
        m1, m2 = R.block_mask(cfg.nc, cfg.na, cfg.nv)
        N1 = R.ric_update(T1, r1, D1, s) * m1
        N2 = R.ric_update(T2, r2, D2, s) * m2
        for got, want in ((b1, N1), (b2, N2)):
            assert np.abs(got.cpu().numpy() - want).max() <= 1e-14 * np.abs(want).max()
        want2 = float(np.sum((N1 - T1) ** 2) + np.sum((N2 - T2) ** 2))
        assert abs(nb2 - want2) <= 1e-12 * want2
        ctx.close()
