"""Host-side logic that needs no GPU: the benchmark's flop count, argument checks and traffic gate, and the DIIS extrapolation."""
import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_plan_flops_counts_contractions_dfc_and_ladder(tmp_path):
    import bench
    plan = tmp_path / "plan.txt"
    plan.write_text("\n".join([
        "SECTION residual",
        "CONTRACT 1/1 R2:HHPP:0,1,2,3 T2:HHPP:0,1,4,5 t0:PPPP:4,5,2,3",      # 2 H^2 P^4
        "DFC 1/1 t1:PP:0,3 B:XPP:X0,0,3 B:XCV:X0,1,2 T1:CV:1,2",             # through the factors
        "LADDER R2 TAU",
        "END",
        "SECTION energy",
        "CONTRACT 1/1 E::: T2:HHPP:0,1,2,3 T2:HHPP:0,1,2,3",
        "END",
    ]) + "\n")
    nc, na, nv, nx = 2, 3, 5, 7
    H, P, C, V = nc + na, na + nv, nc, nv
    total, ladder = bench.plan_flops(nc, na, nv, nx, str(plan))
    c2 = lambda n: n * (n - 1) / 2
    lad = P ** 3 * (P + 1) * nx + 2 * (c2(P + 1) ** 2 * c2(H + 1) + c2(P) ** 2 * c2(H))
    contract = 2.0 * H * H * P ** 4
    # (pq|rs) y with y = T1[1,2]: Z[X] = sum_{1,2} B[X,1,2] T1[1,2], then t1 = sum_X B[X,0,3] Z[X]
    dfc = 2.0 * nx * C * V + 2.0 * nx * P * P
    build = 2.0 * nx * P * P * C * V + 2.0 * P * P * C * V
    assert ladder == lad
    assert total == pytest.approx(contract + min(dfc, build) + lad, rel=1e-12)


class _HostCtx:
    """The two vector calls DIIS makes, on host tensors (stands in for the library here)."""

    def dot(self, a, b):
        return float((a * b).sum())

    def axpby(self, alpha, x, beta, y):
        y.mul_(beta).add_(x, alpha=alpha)


def test_diis_extrapolation_solves_a_linear_fixed_point():
    """For a linear contraction map U(t) = M t + b, DIIS over enough iterates reaches the fixed
    point far faster than plain iteration."""
    from paper_2511_03567_amd.ric import _Diis
    rng = np.random.default_rng(3)
    n = 12
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    M = Q @ np.diag(np.linspace(0.5, 0.98, n)) @ Q.T
    b = rng.standard_normal(n)
    exact = np.linalg.solve(np.eye(n) - M, b)
    to = lambda a: torch.from_numpy(a.copy())

    def run(diis):
        t1, t2 = torch.zeros(1, dtype=torch.float64), torch.zeros(n, dtype=torch.float64)
        acc = _Diis(_HostCtx(), diis) if diis else None
        for it in range(1, 500):
            old = t2.clone()
            t2 = to(M @ t2.numpy() + b)
            step = float((t2 - old).norm())
            if step < 1e-12:
                return it, t2.numpy()
            if acc is not None:
                acc.push((t1.clone(), t2.clone()), (torch.zeros(1, dtype=torch.float64), old - t2))
                acc.extrapolate(t1, t2)
        return None, t2.numpy()

    it_plain, x_plain = run(0)
    it_diis, x_diis = run(n + 2)
    assert it_diis is not None and np.abs(x_diis - exact).max() < 1e-9
    assert it_plain is None or it_diis < it_plain / 4


def test_diis_coefficients_solve_the_constrained_least_squares():
    """ric_diis_coefficients (host code of the library, no GPU): c minimizes |sum c_i e_i| with
    sum c_i = 1; checked against numpy's solution of the bordered system on random error vectors,
    and the fallback to the newest vector when the Gram matrix is singular."""
    import ctypes
    lib_path = os.path.join(ROOT, "paper_2511_03567_amd", "libricmrcc.so")
    if not os.path.exists(lib_path):
        pytest.skip("library not built")
    lib = ctypes.CDLL(lib_path)
    D = ctypes.c_double
    lib.ric_diis_coefficients.argtypes = [ctypes.POINTER(D), ctypes.c_int, ctypes.POINTER(D)]
    lib.ric_diis_coefficients.restype = ctypes.c_int
    rng = np.random.default_rng(5)
    for m in (2, 3, 6, 8):
        E = rng.standard_normal((m, 40))
        G = E @ E.T
        c = (D * m)()
        assert lib.ric_diis_coefficients((D * (m * m))(*G.reshape(-1)), m, c) == 0
        A = np.zeros((m + 1, m + 1))
        A[:m, :m] = G
        A[m, :m] = A[:m, m] = 1.0
        want = np.linalg.solve(A, np.r_[np.zeros(m), 1.0])[:m]
        assert np.allclose(list(c), want, rtol=1e-10, atol=1e-12)
        assert abs(sum(c) - 1.0) < 1e-12
    G = np.ones((3, 3))            # three identical error vectors: singular
    c = (D * 3)()
    assert lib.ric_diis_coefficients((D * 9)(*G.reshape(-1)), 3, c) == 0
    assert list(c) == [0.0, 0.0, 1.0]
    assert lib.ric_diis_coefficients((D * 1)(1.0), 0, c) != 0


def test_sorted_tuple_rdms_equal_ordered_tuple_rdms():
    """The spin-free RDM builder over increasing spin-orbital tuples (with the sorting sign) equals
    the one over every ordered tuple, on dense and sparse CAS vectors."""
    import synthetic as S
    rng = np.random.default_rng(9)
    for na, frac in ((1, 1.0), (3, 1.0), (5, 1.0), (7, 0.1)):
        d, c = S.random_ci(rng, na, frac)
        for a, b in zip(S.spinfree_rdms(d, c, na, 3), S.spinfree_rdms_ordered(d, c, na, 3)):
            assert np.abs(a - b).max() < 1e-14


def test_bench_refuses_several_gpus_and_bad_step_counts():
    """bench.py runs on one GPU: --gpus N > 1 and empty step counts exit with a message before any
    device work."""
    import subprocess
    for argv, word in ((["--gpus", "2"], "one GPU"), (["--steps", "0"], "--steps")):
        p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")] + argv, capture_output=True,
                           text=True, timeout=120, cwd=ROOT)
        assert p.returncode == 2, (argv, p.stderr)
        assert word in p.stderr
        assert p.stdout == ""


def test_bench_reports_ladder_traffic_only_for_the_counted_state(monkeypatch):
    """The ladder's HBM bytes come from counter passes on one state of the kernel sources: the line
    carries them only for that workload and while gemm.hip, kernels.hip and runtime.hip hash to it."""
    import hashlib
    import bench
    h = hashlib.sha256()
    for f in ("gemm.hip", "kernels.hip", "runtime.hip"):
        with open(os.path.join(ROOT, "paper_2511_03567_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    state = dict(bench.LADDER_TRAFFIC, sources_sha256=h.hexdigest()[:16])
    monkeypatch.setattr(bench, "LADDER_TRAFFIC", state)
    assert bench.ladder_traffic(state["workload"]) == state["bytes"]
    assert bench.ladder_traffic("mixed_cas88") is None
    monkeypatch.setattr(bench, "LADDER_TRAFFIC", dict(state, sources_sha256="0" * 16))
    assert bench.ladder_traffic(state["workload"]) is None
