"""Python binding of the C ABI in include/ricmrcc.h (argument marshalling only).

Every computation runs in the HIP library libricmrcc.so next to this file;
there is no CPU fallback.  Device memory and streams come from PyTorch.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libricmrcc.so")
PLAN_PATH = os.path.join(_HERE, "plan.txt")

RIC_FP64 = 0
RIC_FP32MIX = 1

# term groups of ric_residual
RIC_TERMS_LINEAR = 1
RIC_TERMS_QUADRATIC = 2
RIC_TERMS_LADDER = 4
RIC_TERMS_NONLADDER = 8
RIC_TERMS_ALL = 15

RIC_E_NOCONV = -7   # raised by solve() only: the iteration did not reach the tolerance

_ERRORS = {-1: "RIC_E_ARG", -2: "RIC_E_STATE", -3: "RIC_E_OOM", -4: "RIC_E_HIP",
           -5: "RIC_E_NONFINITE", -6: "RIC_E_PLAN", RIC_E_NOCONV: "RIC_E_NOCONV"}

_lib = None


class Block(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 8), ("rank", ctypes.c_int), ("start", ctypes.c_int * 4),
                ("extent", ctypes.c_int * 4)]


class Layout(ctypes.Structure):
    _fields_ = [("nc", ctypes.c_int), ("na", ctypes.c_int), ("nv", ctypes.c_int), ("naux", ctypes.c_int),
                ("nh", ctypes.c_int), ("np", ctypes.c_int), ("t1_elems", ctypes.c_long), ("t2_elems", ctypes.c_long),
                ("nblocks", ctypes.c_int), ("block", Block * 12)]


class RicError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


def library():
    """Load libricmrcc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is missing: run __graft_entry__.build() first")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    D = ctypes.c_double
    I = ctypes.c_int
    lib.ric_create.argtypes = [ctypes.POINTER(P), I, P, ctypes.c_char_p]
    lib.ric_destroy.argtypes = [P]
    lib.ric_destroy.restype = None
    lib.ric_set_spaces.argtypes = [P, I, I, I, I]
    lib.ric_load_fock.argtypes = [P, P]
    lib.ric_load_df.argtypes = [P, P, I]
    lib.ric_layout.argtypes = [P, ctypes.POINTER(Layout)]
    lib.ric_diis_coefficients.argtypes = [ctypes.POINTER(D), I, ctypes.POINTER(D)]
    lib.ric_load_rdms.argtypes = [P, P, P, P]
    lib.ric_residual.argtypes = [P, P, P, P, P, I, ctypes.c_uint]
    lib.ric_update.argtypes = [P, P, P, P, P, D, ctypes.POINTER(D)]
    lib.ric_update_noalloc.argtypes = [P, P, P, P, P, D, ctypes.POINTER(D)]
    lib.ric_energy.argtypes = [P, P, P, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.ric_ladder.argtypes = [P, P, P, I]
    lib.ric_last_timings.argtypes = [P, ctypes.POINTER(D), ctypes.POINTER(D)]
    lib.ric_adjoint_residual.argtypes = [P] * 9 + [I]
    lib.ric_energy_gradient.argtypes = [P] * 7
    lib.ric_lambda_update.argtypes = [P] * 7 + [D, ctypes.POINTER(D)]
    lib.ric_flow_scale.argtypes = [P, P, P, D, P, P]
    lib.ric_flow_fock_gradient.argtypes = [P] * 7 + [D, P]
    lib.ric_build_fock.argtypes = [P, P, P]
    lib.ric_semicanonicalize.argtypes = [P, P, P]
    lib.ric_vec_dot.argtypes = [P, P, P, ctypes.c_long, ctypes.POINTER(D)]
    lib.ric_vec_axpby.argtypes = [P, D, P, D, P, ctypes.c_long]
    lib.ric_last_error.argtypes = [P]
    lib.ric_last_error.restype = ctypes.c_char_p
    for fn in ("ric_create", "ric_set_spaces", "ric_load_fock", "ric_load_df", "ric_load_rdms",
               "ric_residual", "ric_update", "ric_update_noalloc", "ric_energy", "ric_ladder", "ric_last_timings",
               "ric_adjoint_residual", "ric_energy_gradient", "ric_lambda_update", "ric_flow_scale",
               "ric_flow_fock_gradient", "ric_vec_dot", "ric_vec_axpby", "ric_build_fock",
               "ric_semicanonicalize", "ric_layout", "ric_diis_coefficients"):
        getattr(lib, fn).restype = I
    _lib = lib
    return lib


def _ptr(t, shape, name):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError(f"{name} must be a GPU torch tensor")
    if t.dtype != torch.float64:
        raise TypeError(f"{name} must be float64")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One residual engine on one device and stream (torch.cuda.current_stream() by default)."""

    def __init__(self, device=0, stream=None, plan_path=None):
        self.lib = library()
        self.device = torch.device("cuda", device) if isinstance(device, int) else torch.device(device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        path = (plan_path or PLAN_PATH).encode()
        rc = self.lib.ric_create(ctypes.byref(h), self.device.index or 0,
                                 ctypes.c_void_p(stream.cuda_stream), path)
        if rc != 0:
            raise RicError(rc, "ric_create failed")
        self.h = h
        self.sizes = None

    def close(self):
        if getattr(self, "h", None):
            self.lib.ric_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc):
        if rc != 0:
            raise RicError(rc, self.lib.ric_last_error(self.h).decode())

    # --- set-up -----------------------------------------------------------------------
    def set_spaces(self, nc, na, nv, naux):
        self._check(self.lib.ric_set_spaces(self.h, nc, na, nv, naux))
        self.sizes = (nc, na, nv, naux)
        self.n = nc + na + nv
        self.nH = nc + na
        self.nP = na + nv

    def load_fock(self, f):
        self._check(self.lib.ric_load_fock(self.h, _ptr(f, (self.n, self.n), "f")))

    def load_df(self, B, borrow=False):
        """DF factors; borrow=True uses the tensor in place (it is kept referenced here until the
        next load_df) instead of copying it."""
        self._check(self.lib.ric_load_df(self.h, _ptr(B, (self.sizes[3], self.n, self.n), "B"), int(bool(borrow))))
        self._B_borrowed = B if borrow else None

    def layout(self):
        """The amplitude classes of the dense T1/T2 layout: {name: (rank, starts, extents)}."""
        out = Layout()
        self._check(self.lib.ric_layout(self.h, ctypes.byref(out)))
        blocks = {}
        for b in out.block[:out.nblocks]:
            r = 2 * b.rank
            blocks[b.name.decode()] = (b.rank, tuple(b.start[:r]), tuple(b.extent[:r]))
        return blocks

    def load_rdms(self, G1, G2, G3):
        na = self.sizes[1]
        self._check(self.lib.ric_load_rdms(
            self.h, _ptr(G1, (na,) * 2, "G1"), _ptr(G2, (na,) * 4, "G2"), _ptr(G3, (na,) * 6, "G3")))

    # --- hot path ---------------------------------------------------------------------
    def amplitude_shapes(self):
        return (self.nH, self.nP), (self.nH, self.nH, self.nP, self.nP)

    def residual(self, T1, T2, R1, R2, precision=RIC_FP64, terms=RIC_TERMS_ALL):
        s1, s2 = self.amplitude_shapes()
        self._check(self.lib.ric_residual(self.h, _ptr(T1, s1, "T1"), _ptr(T2, s2, "T2"),
                                          _ptr(R1, s1, "R1"), _ptr(R2, s2, "R2"), int(precision), int(terms)))

    def update(self, T1, T2, R1, R2, s):
        s1, s2 = self.amplitude_shapes()
        out = ctypes.c_double()
        self._check(self.lib.ric_update(self.h, _ptr(T1, s1, "T1"), _ptr(T2, s2, "T2"), _ptr(R1, s1, "R1"),
                                        _ptr(R2, s2, "R2"), float(s), ctypes.byref(out)))
        return out.value

    def update_noalloc(self, T1, T2, R1, R2, s):
        """ric_update without any device allocation (scratch in the library's static array)."""
        s1, s2 = self.amplitude_shapes()
        out = ctypes.c_double()
        self._check(self.lib.ric_update_noalloc(self.h, _ptr(T1, s1, "T1"), _ptr(T2, s2, "T2"), _ptr(R1, s1, "R1"),
                                                _ptr(R2, s2, "R2"), float(s), ctypes.byref(out)))
        return out.value

    def energy(self, T1, T2):
        s1, s2 = self.amplitude_shapes()
        e = ctypes.c_double()
        e0 = ctypes.c_double()
        self._check(self.lib.ric_energy(self.h, _ptr(T1, s1, "T1"), _ptr(T2, s2, "T2"), ctypes.byref(e),
                                        ctypes.byref(e0)))
        return e.value, e0.value

    def ladder(self, tau, R2, precision=RIC_FP64):
        _, s2 = self.amplitude_shapes()
        self._check(self.lib.ric_ladder(self.h, _ptr(tau, s2, "tau"), _ptr(R2, s2, "R2"), int(precision)))

    # --- adjoint -----------------------------------------------------------------------
    def adjoint_residual(self, T1, T2, X1, X2, dT1, dT2, dF=None, dB=None, accumulate=False):
        """dT = (dr/dT)^T x; with dF, dB also (dr/df)^T x and (dr/dB)^T x (added to dF, dB when
        accumulate is true)."""
        s1, s2 = self.amplitude_shapes()
        n, nx = self.n, self.sizes[3]
        self._check(self.lib.ric_adjoint_residual(
            self.h, _ptr(T1, s1, "T1"), _ptr(T2, s2, "T2"), _ptr(X1, s1, "X1"), _ptr(X2, s2, "X2"),
            _ptr(dT1, s1, "dT1"), _ptr(dT2, s2, "dT2"), _ptr(dF, (n, n), "dF"), _ptr(dB, (nx, n, n), "dB"),
            int(bool(accumulate))))

    def energy_gradient(self, T1, T2, dT1, dT2, dF, dB):
        s1, s2 = self.amplitude_shapes()
        n, nx = self.n, self.sizes[3]
        self._check(self.lib.ric_energy_gradient(
            self.h, _ptr(T1, s1, "T1"), _ptr(T2, s2, "T2"), _ptr(dT1, s1, "dT1"), _ptr(dT2, s2, "dT2"),
            _ptr(dF, (n, n), "dF"), _ptr(dB, (nx, n, n), "dB")))

    def lambda_update(self, L1, L2, G1, G2, J1, J2, s):
        s1, s2 = self.amplitude_shapes()
        out = ctypes.c_double()
        self._check(self.lib.ric_lambda_update(
            self.h, _ptr(L1, s1, "L1"), _ptr(L2, s2, "L2"), _ptr(G1, s1, "G1"), _ptr(G2, s2, "G2"),
            _ptr(J1, s1, "J1"), _ptr(J2, s2, "J2"), float(s), ctypes.byref(out)))
        return out.value

    def flow_scale(self, L1, L2, s, O1, O2):
        s1, s2 = self.amplitude_shapes()
        self._check(self.lib.ric_flow_scale(self.h, _ptr(L1, s1, "L1"), _ptr(L2, s2, "L2"), float(s),
                                            _ptr(O1, s1, "O1"), _ptr(O2, s2, "O2")))

    def flow_fock_gradient(self, T1, T2, R1, R2, L1, L2, s, dF):
        s1, s2 = self.amplitude_shapes()
        self._check(self.lib.ric_flow_fock_gradient(
            self.h, _ptr(T1, s1, "T1"), _ptr(T2, s2, "T2"), _ptr(R1, s1, "R1"), _ptr(R2, s2, "R2"),
            _ptr(L1, s1, "L1"), _ptr(L2, s2, "L2"), float(s), _ptr(dF, (self.n, self.n), "dF")))

    def build_fock(self, h, f):
        """Generalized Fock matrix f from h with the loaded DF factors and RDMs (not loaded)."""
        self._check(self.lib.ric_build_fock(self.h, _ptr(h, (self.n, self.n), "h"), _ptr(f, (self.n, self.n), "f")))

    def semicanonicalize(self):
        """Rotate the loaded f, B and RDMs to semicanonical orbitals; returns (U, f')."""
        U = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        f = torch.empty_like(U)
        self._check(self.lib.ric_semicanonicalize(self.h, _ptr(U, U.shape, "U"), _ptr(f, f.shape, "f")))
        return U, f

    # --- vector operations (DIIS) --------------------------------------------------------
    def dot(self, a, b):
        if a.shape != b.shape:
            raise ValueError("shape mismatch")
        out = ctypes.c_double()
        self._check(self.lib.ric_vec_dot(self.h, _ptr(a, a.shape, "a"), _ptr(b, b.shape, "b"), a.numel(),
                                         ctypes.byref(out)))
        return out.value

    def axpby(self, alpha, x, beta, y):
        if x.shape != y.shape:
            raise ValueError("shape mismatch")
        self._check(self.lib.ric_vec_axpby(self.h, float(alpha), _ptr(x, x.shape, "x"), float(beta),
                                           _ptr(y, y.shape, "y"), y.numel()))

    def timings(self):
        a = ctypes.c_double()
        b = ctypes.c_double()
        self._check(self.lib.ric_last_timings(self.h, ctypes.byref(a), ctypes.byref(b)))
        return a.value, b.value


def masks(nc, na, nv, device):
    """Boolean masks of the stored amplitudes (all-active blocks excluded)."""
    nH, nP = nc + na, na + nv
    m1 = torch.ones((nH, nP), dtype=torch.bool, device=device)
    m1[nc:, :na] = False
    m2 = torch.ones((nH, nH, nP, nP), dtype=torch.bool, device=device)
    m2[nc:, nc:, :na, :na] = False
    return m1, m2


def diis_coefficients(G):
    """ric_diis_coefficients: weights c with sum c_i = 1 minimizing |sum c_i e_i|, from the
    Gram matrix G[i][j] = <e_i, e_j> (host code of the library; needs no device)."""
    m = int(G.shape[0])
    Gc = (ctypes.c_double * (m * m))(*[float(x) for x in np.asarray(G, dtype=np.float64).reshape(-1)])
    cc = (ctypes.c_double * m)()
    rc = library().ric_diis_coefficients(Gc, m, cc)
    if rc != 0:
        raise RicError(rc, f"ric_diis_coefficients: m = {m}")
    return list(cc)


class _Diis:
    """Pulay's direct inversion in the iterative subspace over amplitude pairs (T1, T2).

    Keeps the last `size` updated amplitudes U_i and their steps e_i = U_i - T_i; the
    extrapolation is sum c_i U_i with sum c_i = 1 minimizing |sum c_i e_i|.
    """

    def __init__(self, ctx: Context, size):
        self.ctx = ctx
        self.size = size
        self.U = []
        self.E = []
        self.B = np.zeros((0, 0))

    def reset(self):
        self.U, self.E, self.B = [], [], np.zeros((0, 0))

    def push(self, U, E):
        if len(self.U) == self.size:
            self.U.pop(0)
            self.E.pop(0)
            self.B = self.B[1:, 1:]
        self.U.append(U)
        self.E.append(E)
        m = len(self.E)
        row = [sum(self.ctx.dot(a, b) for a, b in zip(E, self.E[j])) for j in range(m)]
        B = np.zeros((m, m))
        B[:m - 1, :m - 1] = self.B
        B[m - 1, :] = row
        B[:, m - 1] = row
        self.B = B

    def extrapolate(self, T1, T2):
        m = len(self.U)
        if m < 2:
            return False
        c = diis_coefficients(self.B)
        for T, k in ((T1, 0), (T2, 1)):
            for j in range(m):
                self.ctx.axpby(c[j], self.U[j][k], 0.0 if j == 0 else 1.0, T)
        return True


def solve(ctx: Context, s, tol=1e-8, max_iter=200, precision=RIC_FP64, polish_tol=None, T1=None, T2=None,
          log=None, diis=0, diis_start=2):
    """Regularized iteration (eq. ric-update) from T = 0 until ||t_new - t||_2 < tol.

    precision=RIC_FP32MIX: iterate with mixed-precision residuals until the step
    falls below polish_tol (default 1e-6) or stalls, then continue in fp64 to tol.
    diis > 0: accelerate with DIIS over the last `diis` iterates from iteration diis_start on
    (the history restarts when the precision switches).
    Returns (E_corr, E0, T1, T2, iterations).
    """
    s1, s2 = ctx.amplitude_shapes()
    dev = ctx.device
    if T1 is None:
        T1 = torch.zeros(s1, dtype=torch.float64, device=dev)
        T2 = torch.zeros(s2, dtype=torch.float64, device=dev)
    R1 = torch.empty_like(T1)
    R2 = torch.empty_like(T2)
    mode = precision
    switch = polish_tol if polish_tol is not None else 1e-6
    prev = None
    acc = _Diis(ctx, diis) if diis > 0 else None
    for it in range(1, max_iter + 1):
        if acc is not None:
            P1, P2 = T1.clone(), T2.clone()
        ctx.residual(T1, T2, R1, R2, mode)
        step = ctx.update(T1, T2, R1, R2, s) ** 0.5
        if log is not None:
            log.append({"iter": it, "step": step, "precision": "fp32mix" if mode == RIC_FP32MIX else "fp64"})
        if mode == RIC_FP32MIX and (step < switch or (prev is not None and step > 0.9 * prev and acc is None)):
            mode = RIC_FP64
            if acc is not None:
                acc.reset()
        elif mode == RIC_FP64 and step < tol:
            e, e0 = ctx.energy(T1, T2)
            return e, e0, T1, T2, it
        prev = step
        if acc is not None:
            ctx.axpby(-1.0, T1, 1.0, P1)      # P = T_old - U: the negated step
            ctx.axpby(-1.0, T2, 1.0, P2)
            acc.push((T1.clone(), T2.clone()), (P1, P2))
            if it >= diis_start:
                acc.extrapolate(T1, T2)
    raise RicError(RIC_E_NOCONV, f"regularized iteration did not converge in {max_iter} iterations")


def solve_lambda(ctx: Context, T1, T2, s, tol=1e-10, max_iter=400, log=None, diis=0):
    """Lagrange multipliers of the converged regularized iteration.

    Iterates L <- dE/dT + Delta phi L + J_r^T(phi L) from L = dE/dT until the step norm
    falls below tol (with DIIS over the last `diis` iterates when diis > 0).
    Returns (L1, L2, dE/df at fixed T, dE/dB at fixed T, iterations).
    """
    s1, s2 = ctx.amplitude_shapes()
    n, nx = ctx.n, ctx.sizes[3]
    dev = T1.device
    z = lambda sh: torch.zeros(sh, dtype=torch.float64, device=dev)
    G1, G2, eF, eB = z(s1), z(s2), z((n, n)), z((nx, n, n))
    ctx.energy_gradient(T1, T2, G1, G2, eF, eB)
    L1, L2 = G1.clone(), G2.clone()
    P1, P2, J1, J2 = z(s1), z(s2), z(s1), z(s2)
    acc = _Diis(ctx, diis) if diis > 0 else None
    for it in range(1, max_iter + 1):
        if acc is not None:
            O1, O2 = L1.clone(), L2.clone()
        ctx.flow_scale(L1, L2, s, P1, P2)
        ctx.adjoint_residual(T1, T2, P1, P2, J1, J2)
        step = ctx.lambda_update(L1, L2, G1, G2, J1, J2, s) ** 0.5
        if log is not None:
            log.append({"iter": it, "step": step})
        if step < tol:
            return L1, L2, eF, eB, it
        if acc is not None:
            ctx.axpby(-1.0, L1, 1.0, O1)
            ctx.axpby(-1.0, L2, 1.0, O2)
            acc.push((L1.clone(), L2.clone()), (O1, O2))
            if it >= 2:
                acc.extrapolate(L1, L2)
    raise RicError(RIC_E_NOCONV, f"Lagrangian iteration did not converge in {max_iter} iterations")


def energy_gradient(ctx: Context, T1, T2, s, tol=1e-10, max_iter=400, diis=0):
    """dE_corr/df and dE_corr/dB at the converged amplitudes T1, T2 (flow parameter s)."""
    L1, L2, dF, dB, _ = solve_lambda(ctx, T1, T2, s, tol, max_iter, diis=diis)
    s1, s2 = ctx.amplitude_shapes()
    dev = T1.device
    P1 = torch.zeros(s1, dtype=torch.float64, device=dev)
    P2 = torch.zeros(s2, dtype=torch.float64, device=dev)
    ctx.flow_scale(L1, L2, s, P1, P2)
    J1, J2 = torch.empty_like(P1), torch.empty_like(P2)
    ctx.adjoint_residual(T1, T2, P1, P2, J1, J2, dF, dB, accumulate=True)   # dE/d(f,B) at fixed T + (dr/d(f,B))^T(phi L)
    R1, R2 = torch.empty_like(P1), torch.empty_like(P2)
    ctx.residual(T1, T2, R1, R2)
    ctx.flow_fock_gradient(T1, T2, R1, R2, L1, L2, s, dF)                    # + the denominators' part
    return dF, dB


class RICEnergy(torch.autograd.Function):
    """E_corr(f, B) of the converged spin-free RIC-MRCCSD iteration, differentiable in f and B.

    forward(f, B, ctx, s, tol): loads f and B into the context (whose spaces and RDMs are
    set), solves the regularized iteration and returns E_corr as a 0-d tensor.  backward
    solves the Lagrange multipliers and returns dE/df and dE/dB; the particle-particle
    ladder is regenerated from B in both directions.
    """

    @staticmethod
    def forward(fctx, f, B, ctx: Context, s: float, tol: float = 1e-10):
        f = f.detach().contiguous()
        B = B.detach().contiguous()
        ctx.load_fock(f)
        ctx.load_df(B)
        e, _, T1, T2, _ = solve(ctx, s, tol=tol)
        fctx.ric = (ctx, s, tol, T1, T2, f, B)
        return torch.tensor(e, dtype=torch.float64, device=f.device)

    @staticmethod
    def backward(fctx, grad):
        ctx, s, tol, T1, T2, f, B = fctx.ric
        ctx.load_fock(f)     # the context may have been used for other inputs since forward
        ctx.load_df(B)
        dF, dB = energy_gradient(ctx, T1, T2, s, tol)
        g = float(grad)
        ctx.axpby(0.0, dF, g, dF)     # chain rule: scale by the incoming gradient, on the device
        ctx.axpby(0.0, dB, g, dB)
        return dF, dB, None, None, None
