// Launchers of the bandwidth-bound kernels (kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

namespace ric {

constexpr int kMaxDims = 8;

// partial sums of the two-pass reductions (dot products, update and Lagrangian norms): every
// caller passes a buffer of this many doubles
constexpr int kReducePartials = 4096;

// Iteration space shared by an output view and an input view: element i of the
// space (row-major over ext) is out[sum x_d so[d]] and in[sum x_d si[d]].
struct Iter {
  int nd = 0;
  long total = 0;
  long ext[kMaxDims] = {0};
  long so[kMaxDims] = {0};
  long si[kMaxDims] = {0};
};

hipError_t strided_copy(const Iter& it, double alpha, const double* in, double beta, double* out, hipStream_t st);
hipError_t strided_copy_f32(const Iter& it, double alpha, const double* in, float* out, hipStream_t st);
hipError_t fill(double* p, long n, double v, hipStream_t st);
hipError_t symmetrize_pairs(double* x, int nh, int np, hipStream_t st);
hipError_t mask_active(double* r1, double* r2, int nc, int na, int nv, hipStream_t st);
// w = spin-summed reference 1-RDM over all orbitals (2 on the core diagonal, Gamma1 on the active block)
hipError_t fock_weights(double* w, int n, int nc, int na, const double* g1, hipStream_t st);
// out[i] += alpha * sum_X B[X][i] d[X], B row-major [nx][n2]
hipError_t column_dot(const double* B, const double* d, int nx, long n2, double alpha, double* out, hipStream_t st);
// x <- scale (x + x^T(pairs)) over [nh][nh][np][np]
hipError_t symmetrize_pairs_scaled(double* x, int nh, int np, double scale, hipStream_t st);
// Lagrangian iteration L <- g + Delta phi(Delta) L + j (stored amplitudes); norm2[0] = ||L_new - L||^2
hipError_t lambda_update(double* l1, double* l2, const double* g1, const double* g2, const double* j1,
                         const double* j2, const double* eps, int nc, int na, int nv, double s, double* partial,
                         double* norm2, hipStream_t st);
// o = phi(Delta) L (zero on the excluded blocks)
hipError_t flow_scale(const double* l1, const double* l2, const double* eps, int nc, int na, int nv, double s,
                      double* o1, double* o2, hipStream_t st);
// df[p,p] += sum L [T phi + (T Delta + R) phi'] dDelta/df_pp
hipError_t flow_fock_gradient(const double* t1, const double* t2, const double* r1, const double* r2,
                              const double* l1, const double* l2, const double* eps, int nc, int na, int nv,
                              double s, double* df, hipStream_t st);
// out[0] += alpha * sum a[i] b[i] (deterministic two-pass); partial needs kReducePartials doubles
hipError_t dot_accumulate(const double* a, const double* b, long n, double alpha, double* out, double* partial,
                          hipStream_t st);
// regularized update of T1, T2 in place; norm2[0] = ||t_new - t||^2; partial needs kReducePartials doubles
hipError_t ric_update_kernel(double* t1, double* t2, const double* r1, const double* r2, const double* eps, int nc,
                             int na, int nv, double s, double* partial, double* norm2, hipStream_t st);
hipError_t fock_diagonal(const double* f, int n, double* eps, hipStream_t st);
// sign convention of eigenvectors: every column of the m x m block u (row stride ld) gets its entry of
// largest magnitude (first on ties) positive
hipError_t column_signs(double* u, int m, long ld, hipStream_t st);
hipError_t check_finite(const double* x, long n, int* flag, hipStream_t st);
hipError_t prepare_cumulants(const double* g1, const double* g2, const double* g3, int na, double* ga, double* ea,
                             double* l2, double* k2, double* l3, double* k3, hipStream_t st);
hipError_t reference_energy(const double* f, int n, const double* I4, int nc, int na, const double* g1,
                            const double* g2, double* out, hipStream_t st);
// pair-packed ladder: tau+/- (k<=l, e>=f / k<l, e>f), W+/- per (c,d) pair, and the scatter to R2
// rows of the packed operands have leading dimensions ldp (+) and ldm (-), padding zero-filled
hipError_t pack_tau(const double* tau, int nh, int np, double* tp, double* tm, long ldp, long ldm, hipStream_t st);
hipError_t pack_tau_f32(const double* tau, int nh, int np, float* tp, float* tm, long ldp, long ldm, hipStream_t st);
hipError_t pack_w(const double* w, int np, int rows, int c1, double* wp, double* wm, long ldp, long ldm,
                  hipStream_t st);
hipError_t pack_w_f32(const float* w, int np, int rows, int c1, float* wp, float* wm, long ldp, long ldm,
                      hipStream_t st);
hipError_t ladder_scatter_pm_add(const double* sp, const double* sm, int nh, int np, int c0, int c1, double* r2,
                                 hipStream_t st);
hipError_t ladder_scatter_add(const double* C, int nh, int np, int c0, int c1, int ncol, double* r2, hipStream_t st);

}  // namespace ric
