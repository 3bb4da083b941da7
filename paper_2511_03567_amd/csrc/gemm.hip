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

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

__device__ inline void mma(d4& c, double a, double b) {
  c = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline void mma(f4& c, float a, float b) {
  c = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Geometry of one kernel instance: BM x BN tile, K slab BK, WM x WN wavefronts of
// 64 x 64 (4 x 4 MFMA tiles of 16 x 16 each).
template <int BM_, int BN_, int BK_, int WM_, int WN_, int MINB_ = 1>
struct Geo {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, MINB = MINB_;
  static constexpr int NT = 64 * WM * WN;
  static constexpr int LDSK = BK + 1;           // padded LDS row (elements)
  static constexpr int KPT = BK < 8 ? BK : 8;   // consecutive k per thread per load
  static constexpr int TPR = BK / KPT;          // threads per row
  static constexpr int RPP = NT / TPR;          // rows per pass
  static constexpr int PA = (BM + RPP - 1) / RPP;
  static constexpr int PB = (BN + RPP - 1) / RPP;
};

template <typename T, typename Gm>
struct Slab {
  T a[Gm::PA][Gm::KPT];
  T b[Gm::PB][Gm::KPT];
};

// VEC: rows of A/B are 16-byte aligned and K is a multiple of the vector width,
// so each thread's run of KPT values is fetched with 16-byte loads.
template <typename T, typename Gm, bool VEC>
__device__ inline void fetch(const T* __restrict__ A, const T* __restrict__ B, long lda, long ldb, int M, int N,
                             int K, int m0, int n0, int k0, int tid, Slab<T, Gm>& s) {
  const int r = tid / Gm::TPR;
  const int kk = (tid % Gm::TPR) * Gm::KPT;
  constexpr int VW = 16 / sizeof(T);
#pragma unroll
  for (int p = 0; p < Gm::PA; ++p) {
    const int row = r + p * Gm::RPP;
    const int gm = m0 + row;
    const bool okr = row < Gm::BM && gm < M;
    if constexpr (VEC) {
#pragma unroll
      for (int j = 0; j < Gm::KPT; j += VW) {
        const int gk = k0 + kk + j;
        if (okr && gk < K) {
          if constexpr (sizeof(T) == 8) {
            const d2v v = *reinterpret_cast<const d2v*>(A + (long)gm * lda + gk);
            s.a[p][j] = v[0];
            s.a[p][j + 1] = v[1];
          } else {
            const f4v v = *reinterpret_cast<const f4v*>(A + (long)gm * lda + gk);
            s.a[p][j] = v[0]; s.a[p][j + 1] = v[1]; s.a[p][j + 2] = v[2]; s.a[p][j + 3] = v[3];
          }
        } else {
#pragma unroll
          for (int q = 0; q < VW; ++q) s.a[p][j + q] = T(0);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < Gm::KPT; ++j) {
        const int gk = k0 + kk + j;
        s.a[p][j] = (okr && gk < K) ? A[(long)gm * lda + gk] : T(0);
      }
    }
  }
#pragma unroll
  for (int p = 0; p < Gm::PB; ++p) {
    const int row = r + p * Gm::RPP;
    const int gn = n0 + row;
    const bool okr = row < Gm::BN && gn < N;
    if constexpr (VEC) {
#pragma unroll
      for (int j = 0; j < Gm::KPT; j += VW) {
        const int gk = k0 + kk + j;
        if (okr && gk < K) {
          if constexpr (sizeof(T) == 8) {
            const d2v v = *reinterpret_cast<const d2v*>(B + (long)gn * ldb + gk);
            s.b[p][j] = v[0];
            s.b[p][j + 1] = v[1];
          } else {
            const f4v v = *reinterpret_cast<const f4v*>(B + (long)gn * ldb + gk);
            s.b[p][j] = v[0]; s.b[p][j + 1] = v[1]; s.b[p][j + 2] = v[2]; s.b[p][j + 3] = v[3];
          }
        } else {
#pragma unroll
          for (int q = 0; q < VW; ++q) s.b[p][j + q] = T(0);
        }
      }
    } else {
#pragma unroll
      for (int j = 0; j < Gm::KPT; ++j) {
        const int gk = k0 + kk + j;
        s.b[p][j] = (okr && gk < K) ? B[(long)gn * ldb + gk] : T(0);
      }
    }
  }
}

template <typename T, typename Gm>
__device__ inline void stash(T* As, T* Bs, int tid, const Slab<T, Gm>& s) {
  const int r = tid / Gm::TPR;
  const int kk = (tid % Gm::TPR) * Gm::KPT;
#pragma unroll
  for (int p = 0; p < Gm::PA; ++p) {
    const int row = r + p * Gm::RPP;
    if (row < Gm::BM) {
#pragma unroll
      for (int j = 0; j < Gm::KPT; ++j) As[row * Gm::LDSK + kk + j] = s.a[p][j];
    }
  }
#pragma unroll
  for (int p = 0; p < Gm::PB; ++p) {
    const int row = r + p * Gm::RPP;
    if (row < Gm::BN) {
#pragma unroll
      for (int j = 0; j < Gm::KPT; ++j) Bs[row * Gm::LDSK + kk + j] = s.b[p][j];
    }
  }
}

// Tile kernel.  Acc is the MFMA accumulator type; for fp32 operands the
// per-slab fp32 result is added into fp64 registers (acc64).
// Site only separates the symbols of call sites that profiles attribute
// (0: general contractions, 1: particle-particle ladder).
template <typename T, typename Acc, typename TC, typename Gm, bool VEC, int Site>
__global__ void __launch_bounds__(Gm::NT, Gm::MINB)
gemm_nt_kernel(int M, int N, int K, double alpha, const T* __restrict__ A, long lda,
               const T* __restrict__ B, long ldb, double beta, TC* __restrict__ C, long ldc,
               long strideA, long strideB, long strideC, int zdiv, int ksplit, long strideP,
               double* __restrict__ partial) {
  constexpr int BM = Gm::BM, BN = Gm::BN, BK = Gm::BK, LDSK = Gm::LDSK;
  __shared__ T As[2][BM * LDSK];
  __shared__ T Bs[2][BN * LDSK];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = (wave / Gm::WN) * 64;
  const int wn = (wave % Gm::WN) * 64;
  // batch: z -> (z / zdiv) selects A, (z % zdiv) selects B, z selects C
  const int zb = blockIdx.z / ksplit;
  const int ks = blockIdx.z % ksplit;
  A += (long)(zb / zdiv) * strideA;
  B += (long)(zb % zdiv) * strideB;
  C += (long)zb * strideC;
  // XCD-aware tile order: consecutive workgroup ids land on different XCDs
  // (round robin over 8), so give each XCD a contiguous run of tiles that walks
  // down M with a fixed N column and keeps that B tile hot in the XCD's L2.
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

  Slab<T, Gm> s;
  int buf = 0;
  if (kbeg < kend) {
    fetch<T, Gm, VEC>(A, B, lda, ldb, M, N, kend, m0, n0, kbeg, tid, s);
    stash<T, Gm>(As[0], Bs[0], tid, s);
  }
  __syncthreads();
  const int row = lane & 15;
  const int kq = lane >> 4;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) fetch<T, Gm, VEC>(A, B, lda, ldb, M, N, kend, m0, n0, k0 + BK, tid, s);
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
      stash<T, Gm>(As[buf ^ 1], Bs[buf ^ 1], tid, s);
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

int g_variant = -1;  // -1: default geometry; >= 0 forces one (benchmarking)

// Sum of split-K partial tiles in a fixed order (deterministic), then alpha/beta.
template <int Site>
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

template <typename T, typename Acc, typename TC, typename Gm, int Site = 0>
hipError_t launch_geo(const GemmArgs& g, const T* A, const T* B, TC* C, hipStream_t st, double* scratch,
                      size_t scratch_elems) {
  constexpr int BM = Gm::BM, BN = Gm::BN;
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  // Split K when there are few tiles, choosing the factor so the workgroups fill whole rounds
  // of the resident slots (256 CUs x 2 workgroups of these geometries): the smallest factor
  // reaching 95 % of the slots in every round, else the best one found.
  int ksplit = 1;
  if (g.K > 0 && sizeof(TC) == sizeof(double)) {
    constexpr long kSlots = 512;
    const long base = (long)tiles * g.batch;
    auto fill = [&](long ks) {
      const long w = base * ks;
      return (double)w / (double)(((w + kSlots - 1) / kSlots) * kSlots);
    };
    if (base < 4 * kSlots) {
      double best = fill(1);
      for (int ks = 2; ks <= 64; ++ks) {
        if ((long)g.K / ks < 512) break;
        if ((size_t)ks * g.batch * g.M * g.N > scratch_elems) break;
        const double e = fill(ks);
        if (e > best + 0.01) {
          best = e;
          ksplit = ks;
        }
        if (best >= 0.95) break;
      }
    }
  }
  while (ksplit > 1 && (long)g.batch * ksplit > 65535) ksplit /= 2;
  if ((long)g.batch * ksplit > 65535) return hipErrorInvalidValue;
  constexpr int VW = 16 / sizeof(T);
  const bool vec = (g.K % VW == 0) && (g.lda % VW == 0) && (g.ldb % VW == 0) &&
                   ((uintptr_t)A % 16 == 0) && ((uintptr_t)B % 16 == 0) && (g.strideA % VW == 0) &&
                   (g.strideB % VW == 0);
  dim3 grid(tiles, 1, g.batch * ksplit);
  const long strideP = (long)g.M * g.N;
  if (vec)
    hipLaunchKernelGGL((gemm_nt_kernel<T, Acc, TC, Gm, true, Site>), grid, dim3(Gm::NT), 0, st, g.M, g.N, g.K, g.alpha, A,
                       g.lda, B, g.ldb, g.beta, C, g.ldc, g.strideA, g.strideB, g.strideC, g.zdiv, ksplit, strideP,
                       scratch);
  else
    hipLaunchKernelGGL((gemm_nt_kernel<T, Acc, TC, Gm, false, Site>), grid, dim3(Gm::NT), 0, st, g.M, g.N, g.K, g.alpha, A,
                       g.lda, B, g.ldb, g.beta, C, g.ldc, g.strideA, g.strideB, g.strideC, g.zdiv, ksplit, strideP,
                       scratch);
  if (ksplit > 1) {
    const long total = (long)g.batch * g.M * g.N;
    const int nb = (int)std::min<long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(splitk_reduce<Site>, dim3(nb), dim3(256), 0, st, g.M, g.N, ksplit, g.batch, g.alpha,
                       g.beta, scratch, strideP, reinterpret_cast<double*>(C), g.ldc, g.strideC);
  }
  return hipGetLastError();
}

using G128x16 = Geo<128, 128, 16, 2, 2>;
using G128x32 = Geo<128, 128, 32, 2, 2>;
using G256x16 = Geo<256, 128, 16, 4, 2>;
using G256sq = Geo<256, 256, 16, 4, 4>;
using G128x16b2 = Geo<128, 128, 16, 2, 2, 2>;
using G128x32b2 = Geo<128, 128, 32, 2, 2, 2>;

template <typename T, typename Acc, typename TC>
hipError_t launch(const GemmArgs& g, const T* A, const T* B, TC* C, hipStream_t st, double* scratch,
                  size_t scratch_elems) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0 && g.beta == 1.0) return hipSuccess;
  if (g.site == 1) {
    // the ladder's products always take the default tile shape of their type
    if constexpr (sizeof(T) == 8) return launch_geo<T, Acc, TC, G128x16b2, 1>(g, A, B, C, st, scratch, scratch_elems);
    else return launch_geo<T, Acc, TC, G128x32, 1>(g, A, B, C, st, scratch, scratch_elems);
  }
  int v = g_variant;
  // measured on gfx950: fp64 best with 128x128x16 tiles at two workgroups per CU,
  // fp32 with 128x128x32 tiles
  if (v < 0) v = sizeof(T) == 8 ? 3 : 1;
  switch (v) {
    case 1: return launch_geo<T, Acc, TC, G128x32>(g, A, B, C, st, scratch, scratch_elems);
    case 2: return launch_geo<T, Acc, TC, G256x16>(g, A, B, C, st, scratch, scratch_elems);
    case 3: return launch_geo<T, Acc, TC, G128x16b2>(g, A, B, C, st, scratch, scratch_elems);
    case 4: return launch_geo<T, Acc, TC, G128x32b2>(g, A, B, C, st, scratch, scratch_elems);
    default: return launch_geo<T, Acc, TC, G128x16>(g, A, B, C, st, scratch, scratch_elems);
  }
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

void gemm_set_variant(int v) { g_variant = v; }

}  // namespace ric
