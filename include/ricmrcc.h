/*
 * ricmrcc.h -- C ABI of the MI355X (gfx950) spin-free RIC-MRCCSD residual engine.
 *
 * The library evaluates, on one GPU, the hot path of one amplitude iteration of
 * spin-free RIC-MRCCSD (Szenes et al., "Efficient Implementation of the
 * Spin-Free Renormalized Internally-Contracted Multireference Coupled Cluster
 * Theory"):
 *   - the many-body residuals r^c_k = Hbar^c_k, r^{cd}_{kl} = Hbar^{cd}_{kl} and the
 *     energy E = Hbar_0 of Hbar = H + [H,T] + 1/2[[H,T],T] (Section 2.2), with the
 *     paper's approximations on the two-fold commutator (Section 2.2: energy terms
 *     with two three-active amplitudes dropped; residual terms with two
 *     active-carrying amplitudes or a two-body cumulant dropped),
 *   - spin-free (Section 2.3): only the alpha (singles) and alpha-beta (doubles)
 *     components are stored and computed,
 *   - two-electron integrals from density fitting, (pq|rs) = sum_P B[P,p,q] B[P,r,s];
 *     integrals with three or four virtual-type indices are never stored,
 *   - the flow-regularized Jacobi update (Section 2.2, eq. ric-update).
 *
 * Orbital spaces (Table 1): core (nc), active (na), virtual (nv), ordered
 * core, active, virtual; n = nc + na + nv.  Hole range H = core + active
 * (nH = nc + na), particle range P = active + virtual (nP = na + nv).
 *
 * Amplitude / residual layout ("dense hole-particle layout", row-major, fp64):
 *   T1[k][c]        k in H, c in P:           t^c_k (alpha spin)            nH*nP
 *   T2[k][l][c][d]  k,l in H, c,d in P:       t^{c dbar}_{k lbar}           nH*nH*nP*nP
 * with T2[k][l][c][d] == T2[l][k][d][c] (spin-free pair symmetry,
 * eq. spinfree-perm-sym).  The excluded all-active blocks (T1 active->active,
 * T2 with all four indices active; Section 2.2) are kept at zero: the library
 * writes zeros there in R1/R2 and never changes them in T1/T2.  The eight
 * doubles excitation classes of Section 3.2 (IJAB, IJTU, TUAB, ITAB, ITUV,
 * IJTA, TUVA, ITUA with its two stored blocks) are sub-blocks of this layout.
 *
 * Pointers: every array argument is a DEVICE pointer on the context's device
 * unless stated otherwise; scalar outputs documented as "host" are host
 * pointers written after the context's stream has been synchronized.
 * All work is enqueued on the stream given to ric_create (NULL = default
 * stream).  A context is not thread-safe; calls that overlap on one context race.
 *
 * Errors: functions return RIC_OK (0) or a negative code; the message of the
 * last error is available from ric_last_error().  No C++ exception crosses
 * the ABI.  There is no CPU fallback: every step runs in the library's HIP kernels.
 *
 * Environment (tuning and diagnostics; none changes what is computed beyond rounding):
 *   RIC_LADDER_BUDGET   elements of the ladder's (ce|df) block built per chunk of c rows
 *                       (default 2.8e9 for the residual, 1.4e9 in the adjoint); read per call
 *   RIC_LOOP_BUDGET     elements per chunk of a chunked plan intermediate (default 1.5e9)
 *   RIC_PAD_MIN_FLOPS   products above this many flops get K padded to the vector width (1e10)
 *   RIC_FP32_MIN_FLOPS  in RIC_FP32MIX, products above this many flops take fp32 operands (1e10)
 *   RIC_PROFILE         1: device time per operation kind (synchronizes after every operation);
 *                       2: also each operation above 20 ms
 *   RIC_PROGRESS        set: one stderr line when each expensive phase of a plan section ends
 * All but RIC_LADDER_BUDGET are read once, at ric_create.
 */
#ifndef RICMRCC_H
#define RICMRCC_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ric_ctx ric_ctx;

enum {
  RIC_OK = 0,
  RIC_E_ARG = -1,       /* bad dimension, null pointer, bad option */
  RIC_E_STATE = -2,     /* call before ric_set_spaces or before the required loads */
  RIC_E_OOM = -3,       /* device allocation failed */
  RIC_E_HIP = -4,       /* a HIP runtime call failed */
  RIC_E_NONFINITE = -5, /* a residual, energy or norm is NaN/Inf */
  RIC_E_PLAN = -6       /* the contraction plan file is missing or malformed */
};

enum { RIC_FP64 = 0, RIC_FP32MIX = 1 };

/* Term groups of the residual (ric_residual's term_mask), so each part can be checked on its own:
 * a mask selects at least one of LINEAR / QUADRATIC and at least one of LADDER / NONLADDER. */
enum {
  RIC_TERMS_LINEAR = 1,      /* H + [H,T] (Section 2.2) */
  RIC_TERMS_QUADRATIC = 2,   /* 1/2 [[H,T],T] with the approximations of Section 2.2 */
  RIC_TERMS_LADDER = 4,      /* the particle-particle ladder sum_{ef} (ce|df) tau[k,l,e,f] of those groups */
  RIC_TERMS_NONLADDER = 8,   /* every other term of those groups */
  RIC_TERMS_ALL = 15
};

/* One amplitude class of Section 3.2 as a sub-block of the dense layout below: dimension i
 * covers [start[i], start[i] + extent[i]) of its range (holes H = core + active in [0, nH),
 * particles P = active + virtual in [0, nP)). */
typedef struct {
  char name[8];     /* "IA", "IT", "TA" (singles); "IJAB", "IJTU", "TUAB", "ITAB", "ITUV", "IJTA", "TUVA",
                       "ITUA1" (T[i,t,u,a] = t^{ua}_{it}), "ITUA2" (T[i,t,a,u] = t^{au}_{it}) (doubles) */
  int rank;         /* 1: block of T1[nH][nP]; 2: block of T2[nH][nH][nP][nP] */
  int start[4];
  int extent[4];    /* unused dimensions 0 */
} ric_block_t;

typedef struct {
  int nc, na, nv, naux, nh, np;
  long t1_elems;    /* nH * nP: length of T1, R1 (and of every singles-shaped argument) */
  long t2_elems;    /* nH * nH * nP * nP: length of T2, R2 */
  int nblocks;      /* 12: the 3 singles and 9 doubles classes.  Every other doubles sub-block is the pair
                       image T2[l][k][d][c] of one of them (kept equal) or the excluded all-active block */
  ric_block_t block[12];
} ric_layout_t;

/* Create a context on `device` using `hip_stream` (a hipStream_t, may be NULL).
 * plan_path: the contraction plan generated from the paper's equations
 * (plan.txt shipped next to the library); NULL selects that default file.
 * Ownership: the context owns all device memory it allocates; release with ric_destroy. */
int ric_create(ric_ctx** ctx, int device, void* hip_stream, const char* plan_path);
void ric_destroy(ric_ctx* ctx);

/* Orbital space sizes (Table 1).  nc, nv >= 0, 0 <= na <= 16, naux >= 1.
 * Resets every loaded quantity. */
int ric_set_spaces(ric_ctx* ctx, int nc, int na, int nv, int naux);

/* Generalized Fock matrix f (Section 2.1), n x n row-major, symmetric; copied.
 * Its diagonal gives the denominators Delta of eq. cc-update. */
int ric_load_fock(ric_ctx* ctx, const double* f);

/* Where each amplitude class of Section 3.2 sits in the T1/T2 arrays (host output), for the
 * spaces set by ric_set_spaces. */
int ric_layout(const ric_ctx* ctx, ric_layout_t* out);

/* Density-fitting factors B[P][p][q], naux x n x n row-major, symmetric in (p,q).
 * borrow = 0: copied.  borrow = 1: the caller's device array is used in place (no second copy, 11.5 GB
 * at 809 orbitals); it must stay alive and unchanged until the next ric_load_df, ric_set_spaces or
 * ric_destroy.  Builds the stored integral blocks with at most two particle indices. */
int ric_load_df(ric_ctx* ctx, const double* B, int borrow);

/* Spin-free RDMs of the active space (Section 2.3.2): G1[t][u] = Gamma^t_u,
 * G2[t][u][v][w] = Gamma^{tu}_{vw}, G3[t][u][v][w][x][y] = Gamma^{tuv}_{wxy}
 * (Gamma^{PQ..}_{RS..} = sum over column spins <a+_P a+_Q .. a_S a_R>); copied.
 * Builds the spin-free two- and three-body cumulants.  May be NULL when na == 0. */
int ric_load_rdms(ric_ctx* ctx, const double* G1, const double* G2, const double* G3);

/* Many-body residuals (Section 2.2) of the amplitudes T1, T2 (layout above):
 * R1 = r^c_k (alpha), R2 = r^{c dbar}_{k lbar}.  precision: RIC_FP64, or
 * RIC_FP32MIX (large contractions with fp32 MFMA operands and fp64 accumulation;
 * cumulant, energy and update work stays fp64).  In RIC_FP32MIX the context keeps fp32 copies
 * of T1, T2, the DF factors and the stored integral blocks (half their size; about 25 GB at 809
 * orbitals) while at least 16 GB of the device stay free; ric_energy and the adjoint calls
 * release them.  term_mask (RIC_TERMS_*): the term groups evaluated, RIC_TERMS_ALL for the
 * residual itself.  R1, R2 are overwritten (the excluded blocks zero, R2 pair-symmetric in
 * every case). */
int ric_residual(ric_ctx* ctx, const double* T1, const double* T2, double* R1, double* R2, int precision,
                 unsigned term_mask);

/* Flow-regularized Jacobi update (eq. ric-update), in place:
 * t <- (t Delta + r) (1 - exp(-s Delta^2)) / Delta, Delta = sum of hole minus
 * particle diagonal Fock elements; the factor is 0 at Delta = 0.
 * step_norm2 (host): sum over stored amplitudes of (t_new - t)^2. */
int ric_update(ric_ctx* ctx, double* T1, double* T2, const double* R1, const double* R2, double s,
               double* step_norm2);

/* Allocation-free variant of ric_update, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Arguments, results, layout and error codes are those of ric_update, computed by the same
 * kernels.  The only scratch it needs (the 4096 partial sums of the step norm's two-pass
 * reduction and the result slot) lives in a fixed 64 KiB device array that the library holds
 * once per GPU from the first ric_create on that GPU until the process ends; the call makes
 * no device allocation and frees nothing.  Every context on one GPU shares that array and it
 * keeps the last call's contents (each call overwrites all it reads), so calls that overlap
 * on one GPU (other threads or streams) race; serialize them.  RIC_E_ARG if the reduction
 * ever needed more than the array holds. */
int ric_update_noalloc(ric_ctx* ctx, double* T1, double* T2, const double* R1, const double* R2, double s,
                       double* step_norm2);

/* Energy (Section 2.2): e_corr (host) = Hbar_0 - E0 with the energy approximation;
 * e0 (host, may be NULL) = <Psi0|H|Psi0>, with h recovered from f (Section 2.1). */
int ric_energy(ric_ctx* ctx, const double* T1, const double* T2, double* e_corr, double* e0);

/* Particle-particle ladder alone (the dominant term of the residual):
 * R2[k][l][c][d] += sum_{e,f in P} (ce|df) tau[k][l][e][f] with (ce|df) built from B
 * block by block; tau must satisfy tau[k][l][e][f] == tau[l][k][f][e].
 * For benchmarking and testing that contraction in isolation. */
int ric_ladder(ric_ctx* ctx, const double* tau, double* R2, int precision);

/* ---- adjoint (vector-Jacobian products) of the path ------------------------------------
 * The converged amplitudes are the fixed point T = U(T) of the update of eq. ric-update,
 * U(T) = (T Delta + r(T)) phi(Delta), phi(D) = (1 - exp(-s D^2)) / D.  The gradient of the
 * correlation energy E(T, f, B) of Section 2.2 with respect to the Fock matrix and the DF
 * factors follows from the Lagrange multipliers L of that fixed point:
 *   L = dE/dT + Delta phi L + J_r^T (phi L)                                  (iteration)
 *   dE/df = dE/df|_T + (dr/df)^T (phi L) + sum L [T phi + (T Delta + r) phi'] dDelta/df
 *   dE/dB = dE/dB|_T + (dr/dB)^T (phi L)
 * The calls below evaluate the pieces; the Python layer (ric.py) runs the iteration.
 * Gradients with respect to the doubles are returned projected on pair-symmetric tensors
 * (the space the amplitudes live in) with the excluded all-active blocks zero.  dB is the
 * gradient with respect to every element B[P][p][q] as used (no (p,q) symmetrization). */

/* J^T x for the residuals: with x = (X1, X2) (layouts of R1, R2; X2 is replaced by its
 * pair-symmetric part, both are masked like the residuals), dT = (dr/dT)^T x and, when
 * dF and dB are not NULL, dF = (dr/df)^T x (n x n), dB = (dr/dB)^T x (naux x n x n).
 * The particle-particle ladder is transposed by rebuilding (ce|df) from B in chunks (for dT)
 * and by forming sum_kl x[k,l,c,d] tau[k,l,e,f] in chunks of c (for dB); neither is stored.
 * dT is overwritten; dF and dB are overwritten (accumulate = 0) or added to (accumulate = 1,
 * e.g. onto the energy gradient).  FP64. */
int ric_adjoint_residual(ric_ctx* ctx, const double* T1, const double* T2, const double* X1, const double* X2,
                         double* dT1, double* dT2, double* dF, double* dB, int accumulate);

/* Gradient of the correlation energy functional of Section 2.2 at fixed amplitudes:
 * dT = dE/dT, dF = dE/df, dB = dE/dB.  Outputs overwritten.  FP64. */
int ric_energy_gradient(ric_ctx* ctx, const double* T1, const double* T2, double* dT1, double* dT2, double* dF,
                        double* dB);

/* One step of the Lagrangian iteration, in place: L <- G + Delta phi(Delta) L + J over the
 * stored amplitudes (Delta, phi as in ric_update; G = dE/dT, J = J_r^T(phi L)).
 * step_norm2 (host, may be NULL): sum of (L_new - L)^2. */
int ric_lambda_update(ric_ctx* ctx, double* L1, double* L2, const double* G1, const double* G2, const double* J1,
                      const double* J2, double s, double* step_norm2);

/* O = phi(Delta) L (zero on the excluded blocks): the cotangent passed to ric_adjoint_residual. */
int ric_flow_scale(ric_ctx* ctx, const double* L1, const double* L2, double s, double* O1, double* O2);

/* dF[p][p] += sum over amplitudes of L [T phi + (T Delta + R) phi'] dDelta/df_pp, the part of
 * dE/df that enters through the denominators (R = r(T) at the converged T).  Accumulates. */
int ric_flow_fock_gradient(ric_ctx* ctx, const double* T1, const double* T2, const double* R1, const double* R2,
                           const double* L1, const double* L2, double s, double* dF);

/* Generalized Fock matrix of the reference (Section 2.1) from the one-electron Hamiltonian:
 * f[p][q] = h[p][q] + sum_rs (pq|rs) D[r][s] - sum_{k in core} (pk|kq)
 *           - 1/2 sum_{t,u in active} Gamma1[t][u] (pu|tq),
 * with D the spin-summed reference 1-RDM (2 on the core diagonal, Gamma1 on the active
 * block) and (pq|rs) from the loaded DF factors.  h, f: n x n row-major device pointers;
 * f is overwritten and not loaded into the context (pass it to ric_load_fock). */
int ric_build_fock(ric_ctx* ctx, const double* h, double* f);

/* Semicanonical orbitals (Section 2.2: the denominators Delta are exact for a Fock matrix
 * that is diagonal within the core, active and virtual blocks).  Diagonalizes those three
 * blocks of the loaded f (rocSOLVER dsyevd on the device), and replaces the loaded f, DF
 * factors and RDMs by their rotated forms: f' = U^T f U, B'[X] = U^T B[X] U, every RDM index
 * rotated by the active block of U.  U (n x n, row-major, block-diagonal orthogonal; column
 * j = new orbital j, eigenvalues ascending within each block, each column's entry of largest
 * magnitude positive) is written to the caller; f_out (n x n, may be NULL) receives f'.
 * Amplitudes of the old orbitals transform with the hole and particle blocks of U. */
int ric_semicanonicalize(ric_ctx* ctx, double* U, double* f_out);

/* ---- vector operations for accelerated iterations (DIIS) ------------------------------
 * The paper converges the amplitude equations with a DIIS-accelerated form of the iteration of
 * eq. cc-update (Section 2.2); these two calls are
 * the device work of that extrapolation: inner products of error vectors and linear
 * combinations of amplitude vectors.  n elements, device pointers, enqueued on the context
 * stream. */

/* out (host) = sum_i a[i] b[i], summed in a fixed order (deterministic). */
int ric_vec_dot(ric_ctx* ctx, const double* a, const double* b, long n, double* out);

/* y <- alpha x + beta y (beta = 0 overwrites y without reading it). */
int ric_vec_axpby(ric_ctx* ctx, double alpha, const double* x, double beta, double* y, long n);

/* Coefficients of a DIIS extrapolation (host arrays, no device work): with the m x m Gram matrix
 * G[i][j] = <e_i, e_j> of the error vectors (row-major, m <= 32), c (length m) minimizes
 * |sum c_i e_i| subject to sum c_i = 1.  If that system is singular to working precision, c selects
 * the newest vector (c[m-1] = 1).  RIC_E_ARG for m < 1 or m > 32. */
int ric_diis_coefficients(const double* G, int m, double* c);

/* Milliseconds spent in the ladder during the last ric_residual/ric_ladder call,
 * measured with HIP events on the context stream (host output). */
int ric_last_timings(const ric_ctx* ctx, double* ladder_ms, double* total_ms);

const char* ric_last_error(const ric_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* RICMRCC_H */
