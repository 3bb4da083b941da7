"""Benchmark: seconds per spin-free RIC-MRCCSD residual iteration on one MI355X.

Workload: the 809-orbital CAS(12,12) shape (40 core, 12 active, 757 virtual
orbitals, 2200 auxiliary DF functions) with seeded synthetic inputs.  A step is
one pass of the hot path: the many-body residual (every term, including the
on-the-fly particle-particle ladder) followed by the flow-regularized update and
its norm, in FP64.  After the timed FP64 steps the FP32-mixed residual is timed
once at the amplitudes the first timed step started from, and compared with that
step's FP64 residual.

A step at this size takes about a minute, so the run keeps to a wall-clock budget
(--time-budget, counted from the start of the process): after the first step it
runs at most one warmup step and as many of the requested timed steps as fit, at
least one, leaving room for the mixed residual, the energy and the CPU baseline.
The JSON line reports the steps actually run next to the requested ones.

Prints one JSON line (keys below).  Progress goes to stderr.
"""
import time

T_START = time.perf_counter()

import argparse  # noqa: E402
import json  # noqa: E402
import math  # noqa: E402
import os  # noqa: E402
import sys  # noqa: E402

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6      # TFLOP/s, dense MFMA
PEAK_FP32 = 157.3
PEAK_HBM = 8000.0     # GB/s
METRIC = "s/residual-iteration & TFLOP/s, 809-orb CAS(12,12); FP32-mixed vs FP64 at 1e-6 Eh"

# HBM bytes of one ladder call at the 809-orbital shape, from FETCH_SIZE / WRITE_SIZE passes
# (profiles/ladder_b12_cas1212_hbm_counters.md), scaled by the copy-kernel calibration.  Valid
# only for the kernel and runtime sources they were taken on (the runtime sets the ladder's
# chunking); any change to them reports null.
# flops of one residual at the 809-orbital shape held fixed (the plan's executed count before
# operand pre-combination), so that TFLOP/s against it follows s/iteration as the plan changes
FIXED_FLOPS = {"b12_cas1212": 4.397209499209308e15}

LADDER_TRAFFIC = {"bytes": 7.1152e+13, "sources_sha256": "08543e8f6f8399d3", "workload": "b12_cas1212"}


def log(msg):
    print(f"[bench {time.perf_counter() - T_START:6.1f} s] {msg}", file=sys.stderr, flush=True)


def elapsed():
    return time.perf_counter() - T_START


def _dfc_flops(out, l1, l2, y, ext):
    """Flops of out += sum (pr|qs) y as the runtime executes it: the cheaper of building the
    integral block from the DF factors and going through the factors (Z = L.y, then L.Z)."""
    vol = lambda labs: math.prod(ext[l] for l in set(labs))
    nx = ext[l1[0]]
    eri = l1[1:] + l2[1:]
    best = 2.0 * nx * vol(eri) + 2.0 * vol(eri + y + out)
    for la, lb in ((l1, l2), (l2, l1)):
        zl = [lb[0]]
        ok = True
        for l in lb[1:]:
            summed = l in y and l not in out and l not in la
            if summed:
                continue
            if l in y:
                ok = False
            zl.append(l)
        zl += [l for l in y if l not in lb]
        ok = ok and not any(l in la and l in out for l in zl[1:])
        ok = ok and all(l in la or l in zl for l in out)
        if not ok or vol(zl) > 2.0e9:
            continue
        f = 2.0 * nx * vol([l for l in lb + y if l != lb[0]]) + 2.0 * nx * vol([l for l in la + zl if l != lb[0]])
        best = min(best, f)
    return best


def ladder_flops(nh, n_part, naux):
    """Flops of the pair-packed ladder over a particle range of n_part orbitals: the W build
    over pairs c >= d, n^3 (n + 1) naux, plus the contraction with the (+/-) packed amplitudes,
    2 [C(n+1,2)^2 C(nh+1,2) + C(n,2)^2 C(nh,2)]."""
    c2 = lambda m: m * (m - 1) / 2
    return (n_part ** 3 * (n_part + 1) * naux
            + 2 * (c2(n_part + 1) ** 2 * c2(nh + 1) + c2(n_part) ** 2 * c2(nh)))


def plan_flops(nc, na, nv, naux, plan_path, section="residual"):
    """Flops one evaluation of a plan section executes.

    Binary contractions: 2 * product of the extents of all their indices.  DF terms
    (pr|qs) y: the cheaper of building the block from B plus the contraction and the
    factored route, as the runtime chooses.  Ladder: W build over pairs c >= d plus the
    contraction with the pair-packed (+/-) amplitudes over the particle range P = A + V
    that the runtime runs it on.  Returns (total, ladder).
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
            if sec != section:
                continue
            if t[0] in ("CONTRACT", "CONTRACT0", "DFC"):
                rng = {}
                labs_of = []
                for opd in t[2:]:
                    _, r, labs = opd.split(":")
                    ls = labs.split(",") if labs else []
                    labs_of.append(ls)
                    for x, lab in zip(r, ls):
                        rng[lab] = ext[x]
                if t[0] == "DFC":
                    total += _dfc_flops(labs_of[0], labs_of[1], labs_of[2], labs_of[3], rng)
                else:
                    total += 2.0 * math.prod(rng.values())
            elif t[0] == "LADDER":
                lad = ladder_flops(nc + na, na + nv, naux)
                ladder += lad
                total += lad
    return total, ladder


def ladder_traffic(config):
    import hashlib
    csrc = os.path.join(ROOT, "paper_2511_03567_amd", "csrc")
    h = hashlib.sha256()
    for f in ("gemm.hip", "kernels.hip", "runtime.hip"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    ok = h.hexdigest()[:16] == LADDER_TRAFFIC["sources_sha256"] and config == LADDER_TRAFFIC["workload"]
    return LADDER_TRAFFIC["bytes"] if ok else None


# shapes (nc, na, nv, naux) the oracle is timed on; nc : nv : naux follow the benchmark's
# 40 : 757 : 2200 roughly, with a 4-orbital active space
CPU_SAMPLES = [(2, 4, 16, 40), (3, 4, 24, 60), (4, 4, 32, 80), (5, 4, 40, 100)]


def cpu_baseline(cfg):
    """The oracle timed on a bounded sample: its residual + update at four small shapes,
    a power law t = a N^b fitted in the ladder's size measure N = nH^2 nP^4, extrapolated to
    the benchmark shape (labelled as such)."""
    import numpy as np

    import synthetic as S
    from oracle import ricmrcc as R

    R.term_lists()
    samples = []
    for nc, na, nv, nx in CPU_SAMPLES:
        c = S.custom_config("sample", nc, na, nv, nx, 21)
        inp = S.make_inputs(c)
        ref = R.Reference(nc, na, nv, inp.f, inp.B, inp.G1, inp.G2, inp.G3)
        rng = np.random.default_rng(1)
        m1, m2 = R.block_mask(nc, na, nv)
        nH, nP = nc + na, na + nv
        T1 = rng.standard_normal((nH, nP)) * 0.01 * m1
        T2 = rng.standard_normal((nH, nH, nP, nP)) * 0.01
        T2 = 0.5 * (T2 + T2.transpose(1, 0, 3, 2)) * m2
        t0 = time.perf_counter()
        R1, R2 = ref.residual(T1, T2)
        D1, D2 = R.denominators(inp.f, nc, na, nv)
        R.ric_update(T1, R1, D1, 0.5)
        R.ric_update(T2, R2, D2, 0.5)
        el = time.perf_counter() - t0
        samples.append({"nc": nc, "na": na, "nv": nv, "naux": nx, "s": round(el, 3),
                        "N": float(nH ** 2 * nP ** 4)})
        log(f"oracle sample nc={nc} na={na} nv={nv} naux={nx}: {el:.2f} s")
    x = np.log([s["N"] for s in samples])
    y = np.log([s["s"] for s in samples])
    b, a = np.polyfit(x, y, 1)
    n_full = float((cfg.nc + cfg.na) ** 2 * (cfg.na + cfg.nv) ** 4)
    value = float(math.exp(a + b * math.log(n_full)))
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((l.split(":", 1)[1].strip() for l in fh if l.startswith("model name")), "")
    except OSError:
        pass
    return {
        "value": value,
        "unit": "s/residual-iteration",
        "cores": min(threads, os.cpu_count() or 1),
        "kind": "oracle",
        "sample": ("oracle residual + update timed at (nc, na, nv, naux) = "
                   + ", ".join(f"({s['nc']},{s['na']},{s['nv']},{s['naux']}): {s['s']} s" for s in samples)
                   + f" on {model}; power law t = a N^b in N = nH^2 nP^4 fitted over the four (b = {b:.3f}), "
                     f"extrapolated to N = {n_full:.3e} at the benchmark shape"),
        "fit_exponent": float(b),
        "samples": samples,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0)
    ap.add_argument("--config", default="b12_cas1212")
    ap.add_argument("--time-budget", type=float, default=540.0,
                    help="wall-clock seconds from process start the run keeps to (at least one step runs)")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP32-mixed timing")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--converge", action="store_true",
                    help="also run converged FP32-mixed and FP64 solves at CAS(8,8) and compare energies")
    ap.add_argument("--adjoint", action="store_true",
                    help="also time one adjoint-residual evaluation J_r^T x")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this engine has no multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        sys.exit(2)
    os.environ.setdefault("RIC_PROGRESS", "1")
    import numpy as np
    import torch

    import synthetic as S
    from paper_2511_03567_amd import ric

    budget = args.time_budget
    cfg = S.CONFIGS[args.config]
    dev = torch.device("cuda", 0)
    inp = S.make_inputs(cfg)
    log(f"inputs for {cfg.name} generated")
    ctx = ric.Context(0)
    ctx.set_spaces(cfg.nc, cfg.na, cfg.nv, cfg.naux)
    tt = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to(dev)
    ctx.load_fock(tt(inp.f))
    Bd = tt(inp.B)
    ctx.load_df(Bd)
    del Bd
    ctx.load_rdms(tt(inp.G1), tt(inp.G2), tt(inp.G3))
    del inp
    torch.cuda.synchronize()
    log("inputs loaded on the device")
    s1, s2 = ctx.amplitude_shapes()
    # seeded amplitudes of first-order size (std 1e-2), pair-symmetric, all-active block zero
    gen = torch.Generator(device=dev)
    gen.manual_seed(cfg.seed)
    T1 = torch.randn(s1, dtype=torch.float64, device=dev, generator=gen) * 1e-2
    T2 = torch.randn(s2, dtype=torch.float64, device=dev, generator=gen) * 1e-2
    T2.add_(T2.permute(1, 0, 3, 2).contiguous()).mul_(0.5)
    T1[cfg.nc:, :cfg.na] = 0.0
    T2[cfg.nc:, cfg.nc:, :cfg.na, :cfg.na] = 0.0
    T1s, T2s = T1.clone(), T2.clone()          # amplitudes the first timed step starts from
    R1 = torch.empty_like(T1)
    R2 = torch.empty_like(T2)
    F1 = torch.empty_like(T1)                  # residual of the first timed step
    F2 = torch.empty_like(T2)

    # a plain copy of known size (1 GiB read, 1 GiB written), outside the timed region:
    # hardware byte counters of the other kernels are scaled by what they read for it
    ca = torch.ones(1 << 27, dtype=torch.float64, device=dev)
    cb = torch.mul(ca, 1.0)
    torch.cuda.synchronize()
    del ca, cb
    log("amplitudes initialized; calibration copy done (1 GiB read, 1 GiB written)")

    upd_ms = []

    def step(out1, out2):
        ctx.residual(T1, T2, out1, out2, ric.RIC_FP64)
        lm, tm = ctx.timings()
        ea = torch.cuda.Event(enable_timing=True)
        eb = torch.cuda.Event(enable_timing=True)
        ea.record()          # the library works on torch's current stream
        n2 = ctx.update(T1, T2, out1, out2, cfg.s)
        eb.record()
        eb.synchronize()
        upd_ms.append(ea.elapsed_time(eb))
        return lm, tm, n2

    # time left after this point, keeping room for the legs that follow the timed steps
    def reserve(S):
        r = 15.0                                   # JSON line and teardown
        if not args.no_mixed:
            r += 0.9 * S
        r += max(0.2 * S, 15.0)                    # energy functional
        if not args.no_cpu_baseline:
            r += 45.0
        return r

    # first step: a warmup when a timed step still fits after it, else the one timed step
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lm, tm, n2 = step(F1, F2)
    torch.cuda.synchronize()
    S = time.perf_counter() - t0
    log(f"first fp64 step: {S:.1f} s (residual {tm / 1e3:.1f} s, ladder {lm / 1e3:.1f} s), |dt| {math.sqrt(n2):.3e}")
    fits = lambda k: budget - elapsed() - reserve(S) >= 1.05 * S * k
    warm = 0
    ladder_ms = []
    res_ms = []
    if args.warmup >= 1 and fits(1):
        warm = 1
        # further warmups only when every requested timed step still fits after them
        while warm < args.warmup and fits(1 + args.steps):
            step(R1, R2)
            warm += 1
            log(f"warmup step {warm} done")
        T1s.copy_(T1)
        T2s.copy_(T2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = 0
        while k < args.steps and (k == 0 or fits(1)):
            lm, tm, n2 = step(F1, F2) if k == 0 else step(R1, R2)
            ladder_ms.append(lm)
            res_ms.append(tm)
            k += 1
            log(f"fp64 step {k} done: residual {tm / 1e3:.1f} s, ladder {lm / 1e3:.1f} s, |dt| {math.sqrt(n2):.3e}")
        torch.cuda.synchronize()
        steps = k
        dt = (time.perf_counter() - t0) / steps
    else:
        steps = 1
        dt = S
        ladder_ms.append(lm)
        res_ms.append(tm)
    skipped = []
    if steps < args.steps or warm < args.warmup:
        log(f"time budget {budget:.0f} s: ran {warm} warmup and {steps} timed steps "
            f"of the {args.warmup} + {args.steps} requested")

    plan_path = ric.PLAN_PATH
    flops, lflops_exec = plan_flops(cfg.nc, cfg.na, cfg.nv, cfg.naux, plan_path)
    nh = cfg.nc + cfg.na
    lflops = ladder_flops(nh, cfg.nv, cfg.naux)       # algorithmic: the virtual range
    ladder_s = sum(ladder_ms) / 1e3 / steps
    res_s = sum(res_ms) / 1e3 / steps
    out = {
        "metric": METRIC,
        "value": dt,
        "unit": "s/iteration",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warm,
        "steps_requested": args.steps,
        "warmup_requested": args.warmup,
        "time_budget_s": budget,
        "ms_per_step": dt * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"RIC-MRCCSD residual iteration, {cfg.n} orbitals: nc={cfg.nc} CAS({cfg.na},{cfg.na}) "
                               f"nv={cfg.nv} naux={cfg.naux}, sparse 1% CAS vector, flow s={cfg.s}",
                   "global_batch": 1, "parallelism": "single GPU"},
        "residual_s": res_s,
        "tflops": flops / dt / 1e12,
        "plan_flops": flops,
        "tflops_vs_fixed_count": (FIXED_FLOPS[args.config] / dt / 1e12) if args.config in FIXED_FLOPS else None,
        "fixed_flops": FIXED_FLOPS.get(args.config),
        "roofline": {"bound": "mfma",
                     "kernel": "particle-particle ladder (gemm_nt_kernel<double,...,Site=1> W build and +/- products, "
                               "pack_tau/pack_w/ladder_scatter_pm, splitk_reduce<1>)",
                     "achieved": lflops / ladder_s / 1e12 if ladder_s > 0 else None,
                     "peak": PEAK_FP64, "unit": "TFLOP/s",
                     "frac": (lflops / ladder_s / 1e12) / PEAK_FP64 if ladder_s > 0 else None,
                     "traffic": ladder_traffic(args.config), "ladder_s": ladder_s,
                     "algorithmic_flops": lflops, "executed_flops_particle_range": lflops_exec},
        "nonladder": {"s": res_s - ladder_s, "flops": flops - lflops_exec,
                      "tflops": (flops - lflops_exec) / (res_s - ladder_s) / 1e12 if res_s > ladder_s else None},
    }
    # regularized update: reads T and R, writes T (24 B per stored amplitude), HBM-bound
    n_amp = T1.numel() + T2.numel()
    u_s = min(upd_ms) / 1e3
    out["update"] = {"bound": "hbm", "s": u_s, "achieved": 24.0 * n_amp / u_s / 1e9, "peak": PEAK_HBM,
                     "unit": "GB/s", "frac": 24.0 * n_amp / u_s / 1e9 / PEAK_HBM}
    cpu_res = 45.0 if not args.no_cpu_baseline else 0.0
    # the iterate of the timed steps is not needed from here on: return its 12.8 GB x 2
    del T1, T2
    torch.cuda.empty_cache()
    if args.no_mixed:
        skipped.append("fp32mix (--no-mixed)")
    elif budget - elapsed() - cpu_res - max(0.2 * S, 15.0) >= 0.9 * S:
        # FP32-mixed residual at the amplitudes the first timed step started from, against that
        # step's FP64 residual
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.residual(T1s, T2s, R1, R2, ric.RIC_FP32MIX)
        torch.cuda.synchronize()
        mix = time.perf_counter() - t0
        lm, tm = ctx.timings()
        log(f"fp32-mixed residual done: {mix:.1f} s, ladder {lm / 1e3:.1f} s")
        # max |x| as max(max x, -min x), and the difference in place in F: no 12.8 GB temporaries
        amax = lambda x: max(x.max().item(), -x.min().item())
        scale = max(amax(F1), amax(F2))
        F1.sub_(R1)
        F2.sub_(R2)
        diff = max(amax(F1), amax(F2))
        out["fp32mix"] = {"residual_s": mix, "speedup_vs_fp64_residual": res_s / mix,
                          "max_abs_diff_over_max_abs_fp64": diff / scale,
                          "ladder_s": lm / 1e3,
                          "ladder_tflops": lflops / (lm / 1e3) / 1e12 if lm > 0 else None,
                          "ladder_frac_of_fp32_peak": (lflops / (lm / 1e3) / 1e12) / PEAK_FP32 if lm > 0 else None}
    else:
        skipped.append("fp32mix (time budget)")
    del F1, F2
    if budget - elapsed() - cpu_res >= max(0.2 * S, 15.0):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e, e0 = ctx.energy(T1s, T2s)
        out["energy"] = {"s": time.perf_counter() - t0, "e_corr": e, "e0": e0}
        log(f"energy done: {out['energy']['s']:.2f} s")
    else:
        skipped.append("energy (time budget)")
    if args.converge:
        # converged energies, FP32-mixed iterations + FP64 polish against FP64 throughout, at the
        # CAS(8,8) shape (nc=10, nv=120, naux=360; s = 0.5 and 1.0, DIIS over 6 iterates)
        sm = S.CONFIGS["mixed_cas88"]
        si = S.make_inputs(sm)
        cm = ric.Context(0)
        cm.set_spaces(sm.nc, sm.na, sm.nv, sm.naux)
        cm.load_fock(tt(si.f))
        cm.load_df(tt(si.B))
        cm.load_rdms(tt(si.G1), tt(si.G2), tt(si.G3))
        conv = {}
        for sv in (0.5, 1.0):
            e64, _, _, _, i64 = ric.solve(cm, sv, tol=1e-8, diis=6)
            emx, _, _, _, imx = ric.solve(cm, sv, tol=1e-8, diis=6, precision=ric.RIC_FP32MIX)
            conv[f"s={sv}"] = {"e_fp64": e64, "e_fp32mix": emx, "abs_dE": abs(emx - e64), "iterations": [i64, imx]}
            log(f"CAS(8,8) s={sv}: |dE| mixed vs fp64 {abs(emx - e64):.2e} Eh")
        out["fp32mix_vs_fp64_converged_cas88"] = conv
        cm.close()
        del si
    if args.adjoint:
        # one adjoint-residual evaluation with x = R: J_r^T x (the product the Lagrangian
        # iteration repeats), then J_r^T x with the (f, B) parts
        dT1, dT2 = torch.empty_like(T1s), torch.empty_like(T2s)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.adjoint_residual(T1s, T2s, R1, R2, dT1, dT2)
        torch.cuda.synchronize()
        out["adjoint_residual_s"] = time.perf_counter() - t0
        log(f"adjoint residual (J^T x) done: {out['adjoint_residual_s']:.1f} s")
        n, nx = cfg.n, cfg.naux
        dF = torch.empty((n, n), dtype=torch.float64, device=dev)
        dB = torch.empty((nx, n, n), dtype=torch.float64, device=dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.adjoint_residual(T1s, T2s, R1, R2, dT1, dT2, dF, dB)
        torch.cuda.synchronize()
        out["adjoint_residual_with_f_B_s"] = time.perf_counter() - t0
        log(f"adjoint residual with the f and B parts done: {out['adjoint_residual_with_f_B_s']:.1f} s")
        del dT1, dT2, dF, dB
    if args.no_cpu_baseline:
        skipped.append("cpu_baseline (--no-cpu-baseline)")
    elif budget - elapsed() >= 30.0:
        log("timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline(cfg)
    else:
        skipped.append("cpu_baseline (time budget)")
    out["skipped"] = skipped
    out["wall_s"] = elapsed()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
