// Contraction kernels: C[M][N] = alpha * A(M x K) * B(N x K)^T + beta * C (see gemm.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>

namespace ric {

struct GemmArgs {
  int M = 0, N = 0, K = 0;
  double alpha = 1.0, beta = 0.0;
  long lda = 0, ldb = 0, ldc = 0;
  double* C = nullptr;
  int batch = 1;          // number of C matrices
  int zdiv = 1;           // batch z uses A[z / zdiv], B[z % zdiv], C[z]
  long strideA = 0, strideB = 0, strideC = 0;
  int site = 0;           // 1: particle-particle ladder (a separate kernel symbol for profiles)
  bool ta = false;        // A stored K-major: element (m, k) at A[k * lda + m] (else A[m * lda + k])
  bool tb = false;        // B stored K-major: element (n, k) at B[k * ldb + n] (else B[n * ldb + k])
};

// scratch: fp64 workspace for split-K partial tiles (may be null when scratch_elems == 0)
hipError_t gemm_nt_f64(const GemmArgs& g, const double* A, const double* B, hipStream_t st,
                       double* scratch, size_t scratch_elems);
hipError_t gemm_nt_f32(const GemmArgs& g, const float* A, const float* B, hipStream_t st,
                       double* scratch, size_t scratch_elems);

// fp32 operands and fp32 result (fp64 accumulation inside the tile); no split-K
hipError_t gemm_nt_f32_out32(const GemmArgs& g, const float* A, const float* B, float* C, hipStream_t st);

}  // namespace ric
