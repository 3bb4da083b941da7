// Dense contraction kernels for gfx950 (CDNA4): C[M][N] = alpha * A[M][K] * B[N][K]^T + beta * C.
//
// Every binary tensor contraction of the residual is brought to this "NT" form
// (both operands contiguous along the contracted index K), so one MFMA kernel
// serves the ring, hole-hole, integral-build and ladder contractions.
//
// Tiling: a 256-thread workgroup (4 wavefronts of 64 lanes, arranged 2 x 2)
// computes a 128 x 128 tile of C; each wavefront owns 64 x 64 = 4 x 4 MFMA
// tiles of 16 x 16.  K advances in slabs of 16 staged through LDS, double
// buffered: the next slab is fetched from HBM into registers while the MFMAs
// consume the current one.
//
// FP64 path: v_mfma_f64_16x16x4f64 (16x16 tile, 4-deep K step).
// FP32 path (mixed precision): v_mfma_f32_16x16x4f32 on fp32 operands; the
// fp32 tile accumulators are flushed into fp64 accumulators every slab so the
// long K sums of the residual are carried in fp64.
//
// Lane layout of the 16x16x4 MFMAs (64 lanes, measured on gfx950): operand A
// element (i, k) sits in lane i + 16 k, operand B element (k, j) in lane j + 16 k.
// Result element (i, j): fp32 tile in lane j + 16 (i / 4), register i % 4;
// fp64 tile in lane j + 16 (i % 4), register i / 4.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>
#include "gemm.h"

namespace ric {

namespace {

constexpr int BM = 128;
constexpr int BN = 128;
constexpr int BK = 16;
constexpr int LDSK = BK + 1;      // padded row (in elements) of the K-contiguous LDS tiles

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Slab {
  T a[8];
  T b[8];
};

template <typename T>
__device__ inline void fetch(const T* __restrict__ A, const T* __restrict__ B, long lda, long ldb,
                             int M, int N, int K, int m0, int n0, int k0, int tid, Slab<T>& s) {
  // 256 threads load a 128 x 16 slab of A and of B: thread -> (row = tid / 2, 8 consecutive k)
  const int r = tid >> 1;
  const int kk = (tid & 1) * 8;
  const int gm = m0 + r;
  const int gn = n0 + r;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int gk = k0 + kk + j;
    s.a[j] = (gm < M && gk < K) ? A[(long)gm * lda + gk] : T(0);
    s.b[j] = (gn < N && gk < K) ? B[(long)gn * ldb + gk] : T(0);
  }
}

template <typename T>
__device__ inline void stash(T* As, T* Bs, int tid, const Slab<T>& s) {
  const int r = tid >> 1;
  const int kk = (tid & 1) * 8;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    As[r * LDSK + kk + j] = s.a[j];
    Bs[r * LDSK + kk + j] = s.b[j];
  }
}

__device__ inline void mma(d4& c, double a, double b) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline void mma(f4& c, float a, float b) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Tile kernel.  Acc is the MFMA accumulator type; for fp32 operands the
// per-slab fp32 result is added into fp64 registers (acc64).
template <typename T, typename Acc, typename TC>
__global__ void __launch_bounds__(256)
gemm_nt_kernel(int M, int N, int K, double alpha, const T* __restrict__ A, long lda,
               const T* __restrict__ B, long ldb, double beta, TC* __restrict__ C, long ldc,
               long strideA, long strideB, long strideC, int zdiv, int ksplit, long strideP,
               double* __restrict__ partial) {
  __shared__ T As[2][BM * LDSK];
  __shared__ T Bs[2][BN * LDSK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave >> 1) * 64;
  const int wn = (wave & 1) * 64;
  // batch: z -> (z / zdiv) selects A, (z % zdiv) selects B, z selects C
  const int zb = blockIdx.z / ksplit;
  const int ks = blockIdx.z % ksplit;
  A += (long)(zb / zdiv) * strideA;
  B += (long)(zb % zdiv) * strideB;
  C += (long)zb * strideC;
  // XCD-aware tile order: consecutive workgroup ids land on different XCDs, so
  // walk the tile grid in column-major groups to keep neighbouring tiles of A/B
  // resident in the same L2.
  const int tiles_m = (M + BM - 1) / BM;
  const int nx = gridDim.x;
  const int lin = (nx % 8 == 0) ? (int)(blockIdx.x % 8) * (nx / 8) + (int)(blockIdx.x / 8) : (int)blockIdx.x;
  const int m0 = (lin % tiles_m) * BM;
  const int n0 = (lin / tiles_m) * BN;
  // K range of this split
  const int kchunk = ((K + ksplit - 1) / ksplit + BK - 1) / BK * BK;
  const int kbeg = ks * kchunk;
  const int kend = min(K, kbeg + kchunk);

  constexpr bool kMixed = sizeof(T) == 4;
  Acc acc[4][4];
  double acc64[kMixed ? 4 : 1][4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = Acc{0, 0, 0, 0};
      if constexpr (kMixed) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
      }
    }

  Slab<T> s;
  int buf = 0;
  if (kbeg < kend) {
    fetch(A, B, lda, ldb, M, N, kend, m0, n0, kbeg, tid, s);
    stash(As[0], Bs[0], tid, s);
  }
  __syncthreads();
  const int row = lane & 15;
  const int kq = lane >> 4;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) fetch(A, B, lda, ldb, M, N, kend, m0, n0, k0 + BK, tid, s);
    const T* as = As[buf];
    const T* bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = as[(wm + i * 16 + row) * LDSK + kk + kq];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = bs[(wn + j * 16 + row) * LDSK + kk + kq];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) mma(acc[i][j], av[i], bv[j]);
    }
    if constexpr (kMixed) {
      // carry the slab's fp32 partial sums in fp64
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
          acc[i][j] = Acc{0, 0, 0, 0};
        }
    }
    if (more) {
      stash(As[buf ^ 1], Bs[buf ^ 1], tid, s);
      buf ^= 1;
    }
    __syncthreads();
  }
  // epilogue: fp32 result (i, j) in lane j + 16 (i / 4), register i % 4;
  //           fp64 result (i, j) in lane j + 16 (i % 4), register i / 4
  const int ccol = lane & 15;
  const int crow = kMixed ? (lane >> 4) * 4 : (lane >> 4);
  const int rstep = kMixed ? 1 : 4;
  const long ldo = ksplit > 1 ? (long)N : ldc;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gm = m0 + wm + i * 16 + crow + r * rstep;
        const int gn = n0 + wn + j * 16 + ccol;
        if (gm < M && gn < N) {
          double v;
          if constexpr (kMixed) v = acc64[i][j][r];
          else v = acc[i][j][r];
          if (ksplit > 1) {
            partial[(long)blockIdx.z * strideP + (long)gm * ldo + gn] = v;
          } else {
            const long o = (long)gm * ldo + gn;
            C[o] = beta == 0.0 ? (TC)(alpha * v) : (TC)(alpha * v + beta * (double)C[o]);
          }
        }
      }
}

// Sum of split-K partial tiles in a fixed order (deterministic), then alpha/beta.
__global__ void splitk_reduce(int M, int N, int ksplit, int batches, double alpha, double beta,
                              const double* __restrict__ partial, long strideP, double* __restrict__ C,
                              long ldc, long strideC) {
  const long total = (long)batches * M * N;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long zb = t / ((long)M * N);
    const long rem = t % ((long)M * N);
    const int m = (int)(rem / N);
    const int n = (int)(rem % N);
    double s = 0.0;
    for (int k = 0; k < ksplit; ++k) s += partial[(zb * ksplit + k) * strideP + (long)m * N + n];
    double* c = C + zb * strideC + (long)m * ldc + n;
    *c = beta == 0.0 ? alpha * s : alpha * s + beta * *c;
  }
}

template <typename T, typename Acc, typename TC>
hipError_t launch(const GemmArgs& g, const T* A, const T* B, TC* C, hipStream_t st, double* scratch,
                  size_t scratch_elems) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  int ksplit = 1;
  if (g.K > 0) {
    const long blocks = (long)tiles * g.batch;
    while (blocks * ksplit < 1024 && (long)g.K / (ksplit * 2) >= 512) ksplit *= 2;
    while (ksplit > 1 && (size_t)ksplit * g.batch * g.M * g.N > scratch_elems) ksplit /= 2;
    if (sizeof(TC) != sizeof(double)) ksplit = 1;
  }
  if (g.K <= 0) {
    // C = beta * C
    if (g.beta == 1.0) return hipSuccess;
    ksplit = 1;
  }
  while (ksplit > 1 && (long)g.batch * ksplit > 65535) ksplit /= 2;
  if ((long)g.batch * ksplit > 65535) return hipErrorInvalidValue;
  dim3 grid(tiles, 1, g.batch * ksplit);
  const long strideP = (long)g.M * g.N;
  hipLaunchKernelGGL((gemm_nt_kernel<T, Acc, TC>), grid, dim3(256), 0, st, g.M, g.N, g.K, g.alpha, A, g.lda,
                     B, g.ldb, g.beta, C, g.ldc, g.strideA, g.strideB, g.strideC, g.zdiv, ksplit,
                     strideP, scratch);
  if (ksplit > 1) {
    const long total = (long)g.batch * g.M * g.N;
    const int nb = (int)std::min<long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(splitk_reduce, dim3(nb), dim3(256), 0, st, g.M, g.N, ksplit, g.batch, g.alpha,
                       g.beta, scratch, strideP, reinterpret_cast<double*>(C), g.ldc, g.strideC);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t gemm_nt_f64(const GemmArgs& g, const double* A, const double* B, hipStream_t st,
                       double* scratch, size_t scratch_elems) {
  return launch<double, d4, double>(g, A, B, g.C, st, scratch, scratch_elems);
}

hipError_t gemm_nt_f32(const GemmArgs& g, const float* A, const float* B, hipStream_t st,
                       double* scratch, size_t scratch_elems) {
  return launch<float, f4, double>(g, A, B, g.C, st, scratch, scratch_elems);
}

hipError_t gemm_nt_f32_out32(const GemmArgs& g, const float* A, const float* B, float* C, hipStream_t st) {
  return launch<float, f4, float>(g, A, B, C, st, nullptr, 0);
}

}  // namespace ric
