"""GPU solver: the regularized Jacobi iteration (eq. ric-update) in FP64 and FP32-mixed.

FP64 against the oracle's converged energy (tests/golden/oracle_solve.json, written by
make_solve_golden.py from the oracle alone): within 1e-9 E_h.  FP32-mixed iterations
followed by FP64 polishing: within 1e-6 E_h of the oracle / of the FP64 GPU solve.
"""
import json
import os
import time

import numpy as np
import pytest

import synthetic as S

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_solve.json")


def _ctx(cfg):
    from paper_2511_03567_amd import ric
    inp = S.make_inputs(cfg)
    dev = torch.device("cuda", 0)
    ctx = ric.Context(0)
    ctx.set_spaces(cfg.nc, cfg.na, cfg.nv, cfg.naux)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx.load_fock(t(inp.f))
    ctx.load_df(t(inp.B))
    ctx.load_rdms(t(inp.G1), t(inp.G2), t(inp.G3))
    return ctx


def _golden(key="cases"):
    with open(GOLDEN) as fh:
        return json.load(fh).get(key, [])


@pytest.mark.parametrize("case", _golden(), ids=lambda c: f"{c['config']}-s{c['s']}")
def test_solve_matches_oracle(case):
    from paper_2511_03567_amd import ric
    cfg = S.CONFIGS[case["config"]]
    print(f"solve {case['config']} s={case['s']}", flush=True)
    ctx = _ctx(cfg)
    e64, e0, _, _, it64 = ric.solve(ctx, case["s"], tol=case["tol"])
    emx, _, _, _, itmx = ric.solve(ctx, case["s"], tol=case["tol"], precision=ric.RIC_FP32MIX)
    print(f"  fp64 {e64:.12f} ({it64} it)  mixed {emx:.12f} ({itmx} it)  oracle {case['e_corr']:.12f}", flush=True)
    assert abs(e0 - case["e0"]) < 1e-9
    assert abs(e64 - case["e_corr"]) < 1e-9
    assert abs(it64 - case["iterations"]) <= 1
    assert abs(emx - case["e_corr"]) < 1e-6


@pytest.mark.parametrize("case", _golden("diis_cases"), ids=lambda c: f"{c['config']}-s{c['s']}")
def test_diis_solve_matches_oracle_fixed_point(case):
    """Converged E_corr against the oracle's own fixed point (DIIS over the oracle's update,
    make_solve_golden.py --diis): the CAS(8,8) active space with the CAS(8,8) workload's core
    (nc=10) on 40 virtuals (naux=120), and the CAS(6,6) workload (nc=6, nv=60, naux=180).
    FP64 within 1e-8 E_h, FP32-mixed iterations with FP64 polish within 1e-6 E_h."""
    from paper_2511_03567_amd import ric
    cfg = S.custom_config(case["config"], case["nc"], case["na"], case["nv"], case["naux"], case["seed"])
    print(f"DIIS solve {case['config']} s={case['s']}", flush=True)
    ctx = _ctx(cfg)
    t0 = time.perf_counter()
    e64, e0, _, _, it64 = ric.solve(ctx, case["s"], tol=case["tol"], diis=case["diis"])
    t1 = time.perf_counter()
    emx, _, _, _, itmx = ric.solve(ctx, case["s"], tol=case["tol"], diis=case["diis"],
                                   precision=ric.RIC_FP32MIX)
    t2 = time.perf_counter()
    print(f"  fp64 {e64:.12f} ({it64} it, {t1 - t0:.1f} s)  mixed {emx:.12f} ({itmx} it, {t2 - t1:.1f} s)  "
          f"oracle {case['e_corr']:.12f}  |dE| fp64 {abs(e64 - case['e_corr']):.2e} "
          f"mixed {abs(emx - case['e_corr']):.2e}", flush=True)
    assert abs(e0 - case["e0"]) < 1e-9
    assert abs(e64 - case["e_corr"]) < 1e-8
    assert abs(emx - case["e_corr"]) < 1e-6


@pytest.mark.parametrize("s", [0.5, 1.0])
def test_mixed_solve_matches_fp64_cas88(s):
    """CAS(8,8), nc=10, nv=120, naux=360: the large ring terms and the ladder run as FP32 MFMA tiles.

    Where the FP64 iteration converges, the mixed iteration (then FP64 polish) reaches the
    same energy within 1e-6 E_h.  Where it does not (plain regularized Jacobi at larger s),
    the mixed iteration must fail the same way, following the FP64 step norms closely.
    """
    from paper_2511_03567_amd import ric
    cfg = S.CONFIGS["mixed_cas88"]
    print(f"solve mixed_cas88 s={s}", flush=True)
    ctx = _ctx(cfg)
    log64, logmx = [], []
    t0 = time.perf_counter()
    try:
        e64, _, _, _, it64 = ric.solve(ctx, s, tol=1e-8, log=log64)
    except ric.RicError:
        e64 = None
    t1 = time.perf_counter()
    try:
        emx, _, _, _, itmx = ric.solve(ctx, s, tol=1e-8, precision=ric.RIC_FP32MIX, log=logmx)
    except ric.RicError:
        emx = None
    t2 = time.perf_counter()
    nmix = sum(1 for r in logmx if r["precision"] == "fp32mix")
    steps64 = [r["step"] for r in log64]
    print(f"  fp64: {len(log64)} it, {t1 - t0:.1f} s, E {e64}; mixed: {len(logmx)} it ({nmix} mixed), "
          f"{t2 - t1:.1f} s, E {emx}", flush=True)
    print("  fp64 step norms every 20 iterations: " + " ".join(f"{x:.2e}" for x in steps64[::20]), flush=True)
    assert nmix > 0
    if e64 is not None:
        print(f"  |dE| {abs(emx - e64):.2e}", flush=True)
        assert abs(emx - e64) < 1e-6
    else:
        assert emx is None
        n = min(nmix, 10)
        a = np.array(steps64[:n])
        b = np.array([r["step"] for r in logmx[:n]])
        assert np.all(np.abs(a - b) <= 1e-5 * np.abs(a))


def test_diis_matches_oracle_in_fewer_iterations():
    """DIIS over the regularized update reaches the oracle's fixed point (same energy)."""
    from paper_2511_03567_amd import ric
    case = _golden()[0]
    cfg = S.CONFIGS[case["config"]]
    ctx = _ctx(cfg)
    e, _, _, _, it = ric.solve(ctx, case["s"], tol=case["tol"], diis=6)
    print(f"  DIIS {e:.12f} in {it} iterations (plain iteration: {case['iterations']})", flush=True)
    assert abs(e - case["e_corr"]) < 1e-9
    assert it < case["iterations"]


def test_diis_converges_cas88_at_larger_flow():
    """CAS(8,8), s = 1.0, where the plain iteration creeps: DIIS converges, in FP64 and in
    mixed precision with FP64 polish, to the same energy within 1e-6 E_h."""
    from paper_2511_03567_amd import ric
    cfg = S.CONFIGS["mixed_cas88"]
    ctx = _ctx(cfg)
    log64, logmx = [], []
    e64, _, _, _, it64 = ric.solve(ctx, 1.0, tol=1e-8, diis=6, log=log64)
    emx, _, _, _, itmx = ric.solve(ctx, 1.0, tol=1e-8, diis=6, precision=ric.RIC_FP32MIX, log=logmx)
    nmix = sum(1 for r in logmx if r["precision"] == "fp32mix")
    print(f"  DIIS fp64 {e64:.12f} ({it64} it)  mixed {emx:.12f} ({itmx} it, {nmix} mixed)  "
          f"|dE| {abs(emx - e64):.2e}", flush=True)
    assert nmix > 0
    assert abs(emx - e64) < 1e-6


@pytest.mark.timeout(600)
def test_mixed_solve_matches_fp64_cas1414():
    """CAS(14,14) (nc=20, nv=300, naux=900, sparse 1 % CAS vector), s = 0.5, DIIS over 6 iterates:
    FP32-mixed iterations followed by FP64 polish reach the FP64 energy within 1e-6 E_h."""
    from paper_2511_03567_amd import ric
    cfg = S.CONFIGS["large_cas1414"]
    print(f"solve large_cas1414 s={cfg.s}", flush=True)
    t0 = time.perf_counter()
    ctx = _ctx(cfg)
    log64, logmx = [], []
    t1 = time.perf_counter()
    e64, _, _, _, it64 = ric.solve(ctx, cfg.s, tol=1e-8, max_iter=100, diis=6, log=log64)
    t2 = time.perf_counter()
    emx, _, _, _, itmx = ric.solve(ctx, cfg.s, tol=1e-8, max_iter=100, diis=6, precision=ric.RIC_FP32MIX,
                                   log=logmx)
    t3 = time.perf_counter()
    nmix = sum(1 for r in logmx if r["precision"] == "fp32mix")
    print(f"  inputs {t1 - t0:.1f} s; fp64 {e64:.12f} ({it64} it, {t2 - t1:.1f} s); mixed {emx:.12f} "
          f"({itmx} it, {nmix} mixed, {t3 - t2:.1f} s); |dE| {abs(emx - e64):.2e}", flush=True)
    ctx.close()
    assert nmix > 0
    assert abs(emx - e64) < 1e-6
