"""Benchmark: seconds per spin-free RIC-MRCCSD residual iteration on one MI355X.

Workload: the 809-orbital CAS(12,12) shape (40 core, 12 active, 757 virtual
orbitals, 2200 auxiliary DF functions) with seeded synthetic inputs.  A step is
one pass of the hot path: the many-body residual (every term, including the
on-the-fly particle-particle ladder) followed by the flow-regularized update and
its norm.  FP64 is timed first; the FP32-mixed residual is timed after it.

Prints one JSON line (see the keys below).  Progress goes to stderr.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6      # TFLOP/s, dense MFMA
PEAK_FP32 = 157.3
METRIC = "s/residual-iteration & TFLOP/s, 809-orb CAS(12,12); FP32-mixed vs FP64 at 1e-6 Eh"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def plan_flops(nc, na, nv, naux, plan_path):
    """Algorithmic flops of one residual evaluation from the contraction plan.

    Binary contractions: 2 * product of the extents of all their indices.  DF
    blocks (pr|qs) built from B: 2 * naux * product of their extents plus the
    contraction.  Ladder: W build over pairs c >= d plus the contraction with the
    pair-packed (+/-) amplitudes, counted over the particle range P = A + V.
    Returns (total, ladder).
    """
    ext = {"C": nc, "A": na, "V": nv, "H": nc + na, "P": na + nv, "G": nc + na + nv, "X": naux}
    total = 0.0
    ladder = 0.0
    sec = None
    with open(plan_path) as fh:
        for line in fh:
            t = line.split()
            if not t:
                continue
            if t[0] == "SECTION":
                sec = t[1]
                continue
            if sec != "residual":
                continue
            if t[0] in ("CONTRACT", "CONTRACT0", "DFC"):
                rng = {}
                eri = []
                for k, opd in enumerate(t[2:]):
                    _, r, labs = opd.split(":")
                    ls = labs.split(",") if labs else []
                    for x, lab in zip(r, ls):
                        rng[lab] = x
                    if t[0] == "DFC" and k in (1, 2):
                        eri += list(r[1:])
                f = 2.0
                for lab, x in rng.items():
                    if x != "X":
                        f *= ext[x]
                if eri:
                    b = 2.0 * naux
                    for x in eri:
                        b *= ext[x]
                    f += b
                total += f
            elif t[0] == "LADDER":
                nP, nH = na + nv, nc + na
                c2 = lambda n: n * (n - 1) / 2
                lad = nP ** 3 * (nP + 1) * naux + 2 * (c2(nP + 1) ** 2 * c2(nH + 1) + c2(nP) ** 2 * c2(nH))
                ladder += lad
                total += lad
    return total, ladder


def cpu_baseline(flops_full, plan_path):
    """The oracle timed on a bounded sample: its full residual at a small shape, scaled to
    the benchmark shape by the ratio of algorithmic flops."""
    import numpy as np

    import synthetic as S
    from oracle import ricmrcc as R

    nc, na, nv, nx = 4, 4, 40, 60
    cfg = S.custom_config("sample", nc, na, nv, nx, 21)
    inp = S.make_inputs(cfg)
    ref = R.Reference(nc, na, nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
    rng = np.random.default_rng(1)
    m1, m2 = R.block_mask(nc, na, nv)
    nH, nP = nc + na, na + nv
    T1 = rng.standard_normal((nH, nP)) * 0.01 * m1
    T2 = rng.standard_normal((nH, nH, nP, nP)) * 0.01
    T2 = 0.5 * (T2 + T2.transpose(1, 0, 3, 2)) * m2
    R.term_lists()
    t0 = time.perf_counter()
    R1, R2 = ref.residual(T1, T2)
    D1, D2 = R.denominators(inp.f, nc, na, nv)
    R.ric_update(T1, R1, D1, 0.5)
    R.ric_update(T2, R2, D2, 0.5)
    el = time.perf_counter() - t0
    f_sample, _ = plan_flops(nc, na, nv, nx, plan_path)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {
        "value": el * flops_full / f_sample,
        "unit": "s/residual-iteration",
        "cores": min(threads, os.cpu_count() or 1),
        "kind": "oracle",
        "sample": (f"oracle residual + update at nc={nc} na={na} nv={nv} naux={nx} took {el:.2f} s; "
                   f"scaled by algorithmic flops {flops_full:.3e}/{f_sample:.3e} (extrapolated)"),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--config", default="b12_cas1212")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-mixed timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this engine has no multi-GPU path "
              "(the sharding design is described in DESIGN.md)", file=sys.stderr)
        sys.exit(2)
    os.environ.setdefault("RIC_PROGRESS", "1")
    import numpy as np
    import torch

    import synthetic as S
    from paper_2511_03567_amd import ric

    cfg = S.CONFIGS[args.config]
    dev = torch.device("cuda", 0)
    t0 = time.perf_counter()
    inp = S.make_inputs(cfg)
    log(f"inputs for {cfg.name} generated in {time.perf_counter() - t0:.1f} s")
    ctx = ric.Context(0)
    ctx.set_spaces(cfg.nc, cfg.na, cfg.nv, cfg.naux)
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx.load_fock(tt(inp.f))
    Bd = tt(inp.B)
    ctx.load_df(Bd)
    del Bd
    ctx.load_rdms(tt(inp.G1), tt(inp.G2), tt(inp.G3))
    torch.cuda.synchronize()
    log("inputs loaded on the device")
    s1, s2 = ctx.amplitude_shapes()
    T1 = torch.zeros(s1, dtype=torch.float64, device=dev)
    T2 = torch.zeros(s2, dtype=torch.float64, device=dev)
    R1 = torch.empty_like(T1)
    R2 = torch.empty_like(T2)

    def step(prec):
        ctx.residual(T1, T2, R1, R2, prec)
        return ctx.update(T1, T2, R1, R2, cfg.s)

    for w in range(args.warmup):
        step(ric.RIC_FP64)
        log(f"warmup step {w + 1} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ladder_ms = 0.0
    res_ms = 0.0
    for k in range(args.steps):
        n2 = step(ric.RIC_FP64)
        lm, tm = ctx.timings()
        ladder_ms += lm
        res_ms += tm
        log(f"fp64 step {k + 1} done: residual {tm / 1e3:.1f} s, ladder {lm / 1e3:.1f} s, |dt| {math.sqrt(n2):.3e}")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    plan_path = ric.PLAN_PATH
    flops, lflops = plan_flops(cfg.nc, cfg.na, cfg.nv, cfg.naux, plan_path)
    ladder_s = ladder_ms / 1e3 / args.steps
    out = {
        "metric": METRIC,
        "value": dt,
        "unit": "s/iteration",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"RIC-MRCCSD residual iteration, {cfg.n} orbitals: nc={cfg.nc} CAS({cfg.na},{cfg.na}) "
                               f"nv={cfg.nv} naux={cfg.naux}, sparse 1% CAS vector, flow s={cfg.s}",
                   "global_batch": 1, "parallelism": "single GPU"},
        "tflops": flops / dt / 1e12,
        "algorithmic_flops": flops,
        "roofline": {"bound": "mfma", "kernel": "particle-particle ladder (gemm_nt_kernel f64)",
                     "achieved": lflops / ladder_s / 1e12 if ladder_s > 0 else None,
                     "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": (lflops / ladder_s / 1e12) / PEAK_FP64 if ladder_s > 0 else None,
                     "traffic": None, "ladder_s": ladder_s, "ladder_algorithmic_flops": lflops},
    }
    if not args.no_mixed:
        t0 = time.perf_counter()
        ctx.residual(T1, T2, R1, R2, ric.RIC_FP32MIX)
        torch.cuda.synchronize()
        mix = time.perf_counter() - t0
        lm, tm = ctx.timings()
        log(f"fp32-mixed residual done: {mix:.1f} s, ladder {lm / 1e3:.1f} s")
        out["fp32mix_residual_s"] = mix
        out["fp32mix_ladder_tflops"] = lflops / (lm / 1e3) / 1e12 if lm > 0 else None
        out["fp32mix_ladder_frac_of_fp32_peak"] = (lflops / (lm / 1e3) / 1e12) / PEAK_FP32 if lm > 0 else None
    if not args.no_cpu_baseline:
        del inp
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(flops, plan_path)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
