// Dense contraction kernels for gfx950 (CDNA4): C[M][N] = alpha * A(M x K) * B(N x K)^T + beta * C.
//
// Every binary tensor contraction of the residual is brought to this form, so one
// MFMA kernel serves the ring, hole-hole, integral-build and ladder contractions.
// Each operand is read in the layout it already has in HBM:
//   A row-major  [M][K] (K contiguous)  or  A "K-major" [K][M] (M contiguous, ta = true),
//   B row-major  [N][K] (K contiguous)  or  B "K-major" [K][N] (N contiguous, tb = true),
// so a stored block whose contracted indices lead (the integral blocks, read with
// their hole-particle pairs summed) needs no transposed copy.
//
// Tiling: a 256-thread workgroup (4 wavefronts of 64 lanes, arranged 2 x 2)
// computes a tile of C: 128 x 128 in fp64 (each wavefront 64 x 64 = 4 x 4 MFMA tiles of
// 16 x 16, two workgroups per CU), 64 x 128 in fp32 (each wavefront 32 x 64, so the fp64 carry
// of the fp32 partial sums fits three wavefronts per SIMD).  K advances in slabs staged through
// LDS, double buffered:
// the next slab is fetched from HBM into registers while the MFMAs consume the
// current one.  A row-major operand's slab sits in LDS as [row][k] (rows padded by
// one element); a K-major operand's slab as [k][row] (rows padded by two), both
// read by the MFMA loop with 16 consecutive lanes on consecutive LDS words.
//
// FP64 path: v_mfma_f64_16x16x4f64 (16x16 tile, 4-deep K step).
// FP32 path (mixed precision): v_mfma_f32_16x16x4f32 on fp32 operands; the
// fp32 tile accumulators are flushed into fp64 accumulators every 128 terms of K
// (every fourth 32-deep slab, and at the end of the tile's K range) so the long K
// sums of the residual are carried in fp64.  Flushing every slab instead costs
// 6-7 % of the fp32 GEMM rate on gfx950 (the fp64 adds and conversions).
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

// Geometry of one kernel instance: BM x BN tile, K slab BK, WM x WN wavefronts, each owning
// TI x TJ MFMA tiles of 16 x 16.
// CO: K-major operands are read two rows per thread, consecutive threads on consecutive rows
// (one coalesced pass per pair of k), instead of a run of rows per thread.
template <int BM_, int BN_, int BK_, int WM_, int WN_, int MINB_ = 1, int TI_ = 4, int TJ_ = 4, bool CO_ = false>
struct Geo {
  static constexpr int BM = BM_, BN = BN_, BK = BK_, WM = WM_, WN = WN_, MINB = MINB_, TI = TI_, TJ = TJ_;
  static constexpr bool CO = CO_;
  static constexpr int NT = 64 * WM * WN;
  static_assert(BM == WM * 16 * TI && BN == WN * 16 * TJ, "wave tiles");
};

// How the threads of a workgroup load one operand's R x BK slab and where it sits in LDS.
//  TR = false: rows of K contiguous.  Each thread loads KPT consecutive k of one row.
//  TR = true:  K-major ([k][row], rows contiguous).  Each thread loads RPT consecutive rows
//              of one k (RPT = one vector when CO).
template <typename T, int R, int BK, int NT, bool TR, bool CO = false>
struct Tile {
  static constexpr int VW = 16 / (int)sizeof(T);
  // row-major source
  static constexpr int KPT = BK < 8 ? BK : 8;
  static constexpr int TPR = BK / KPT;            // threads per row
  static constexpr int RPP = NT / TPR;            // rows per pass
  static constexpr int PN = (R + RPP - 1) / RPP;  // passes
  static constexpr int LDSK = BK + 1;
  // K-major source
  static constexpr int RPT0 = R * BK / NT;
  static constexpr int RPT = (CO || RPT0 < VW) ? VW : RPT0;   // rows per thread
  static constexpr int TPK = R / RPT;                 // threads per k
  static constexpr int KPP = NT / TPK;                // k per pass
  static constexpr int PT = (BK + KPP - 1) / KPP;     // passes
  static constexpr int LDSR = R + 2;
  static constexpr int E = TR ? PT * RPT : PN * KPT;  // elements held per thread
  static constexpr int LDS = TR ? BK * LDSR : R * LDSK;
  static_assert(!TR || (R % RPT == 0 && RPT % VW == 0), "K-major tile split");
  static_assert(TR || BK % KPT == 0, "row-major tile split");

  // Fetch the slab [k0, k0 + BK) of rows [r0, r0 + R) into registers.  VEC: 16-byte loads
  // (the contiguous extent is a multiple of the vector width and rows are aligned).
  template <bool VEC>
  __device__ static inline void fetch(const T* __restrict__ src, long ld, int nrows, int kend, int r0, int k0,
                                      int tid, T* v) {
    if constexpr (!TR) {
      const int r = tid / TPR;
      const int kk = (tid % TPR) * KPT;
#pragma unroll
      for (int p = 0; p < PN; ++p) {
        const int row = r + p * RPP;
        const int gr = r0 + row;
        const bool okr = row < R && gr < nrows;
#pragma unroll
        for (int j = 0; j < KPT; j += (VEC ? VW : 1)) {
          const int gk = k0 + kk + j;
          if constexpr (VEC) {
            if (okr && gk < kend) {
              if constexpr (sizeof(T) == 8) {
                const d2v x = *reinterpret_cast<const d2v*>(src + (long)gr * ld + gk);
                v[p * KPT + j] = x[0];
                v[p * KPT + j + 1] = x[1];
              } else {
                const f4v x = *reinterpret_cast<const f4v*>(src + (long)gr * ld + gk);
                v[p * KPT + j] = x[0]; v[p * KPT + j + 1] = x[1]; v[p * KPT + j + 2] = x[2]; v[p * KPT + j + 3] = x[3];
              }
            } else {
#pragma unroll
              for (int q = 0; q < VW; ++q) v[p * KPT + j + q] = T(0);
            }
          } else {
            v[p * KPT + j] = (okr && gk < kend) ? src[(long)gr * ld + gk] : T(0);
          }
        }
      }
    } else {
      const int kr = tid / TPK;
      const int rr = (tid % TPK) * RPT;
#pragma unroll
      for (int p = 0; p < PT; ++p) {
        const int k = kr + p * KPP;
        const int gk = k0 + k;
        const bool okk = k < BK && gk < kend;
#pragma unroll
        for (int j = 0; j < RPT; j += (VEC ? VW : 1)) {
          const int gr = r0 + rr + j;
          if constexpr (VEC) {
            if (okk && gr < nrows) {
              if constexpr (sizeof(T) == 8) {
                const d2v x = *reinterpret_cast<const d2v*>(src + (long)gk * ld + gr);
                v[p * RPT + j] = x[0];
                v[p * RPT + j + 1] = x[1];
              } else {
                const f4v x = *reinterpret_cast<const f4v*>(src + (long)gk * ld + gr);
                v[p * RPT + j] = x[0]; v[p * RPT + j + 1] = x[1]; v[p * RPT + j + 2] = x[2]; v[p * RPT + j + 3] = x[3];
              }
            } else {
#pragma unroll
              for (int q = 0; q < VW; ++q) v[p * RPT + j + q] = T(0);
            }
          } else {
            v[p * RPT + j] = (okk && gr < nrows) ? src[(long)gk * ld + gr] : T(0);
          }
        }
      }
    }
  }

  __device__ static inline void stash(T* lds, int tid, const T* v) {
    if constexpr (!TR) {
      const int r = tid / TPR;
      const int kk = (tid % TPR) * KPT;
#pragma unroll
      for (int p = 0; p < PN; ++p) {
        const int row = r + p * RPP;
        if (row < R) {
#pragma unroll
          for (int j = 0; j < KPT; ++j) lds[row * LDSK + kk + j] = v[p * KPT + j];
        }
      }
    } else {
      const int kr = tid / TPK;
      const int rr = (tid % TPK) * RPT;
#pragma unroll
      for (int p = 0; p < PT; ++p) {
        const int k = kr + p * KPP;
        if (k < BK) {
#pragma unroll
          for (int j = 0; j < RPT; ++j) lds[k * LDSR + rr + j] = v[p * RPT + j];
        }
      }
    }
  }

  // element (row, k) of the slab in LDS
  __device__ static inline T at(const T* lds, int row, int k) {
    if constexpr (!TR) return lds[row * LDSK + k];
    else return lds[k * LDSR + row];
  }
};

// Tile kernel.  Acc is the MFMA accumulator type; for fp32 operands the
// per-slab fp32 result is added into fp64 registers (acc64).
// Site only separates the symbols of call sites that profiles attribute
// (0: general contractions, 1: particle-particle ladder).
template <typename T, typename Acc, typename TC, typename Gm, bool VEC, bool TA, bool TB, int Site>
__global__ void __launch_bounds__(Gm::NT, Gm::MINB)
gemm_nt_kernel(int M, int N, int K, double alpha, const T* __restrict__ A, long lda,
               const T* __restrict__ B, long ldb, double beta, TC* __restrict__ C, long ldc,
               long strideA, long strideB, long strideC, int zdiv, int ksplit, long strideP,
               double* __restrict__ partial) {
  constexpr int BM = Gm::BM, BN = Gm::BN, BK = Gm::BK, NT = Gm::NT;
  using TileA = Tile<T, BM, BK, NT, TA, Gm::CO>;
  using TileB = Tile<T, BN, BK, NT, TB, Gm::CO>;
  __shared__ T As[2][TileA::LDS];
  __shared__ T Bs[2][TileB::LDS];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  constexpr int TI = Gm::TI, TJ = Gm::TJ;
  const int wm = (wave / Gm::WN) * (16 * TI);
  const int wn = (wave % Gm::WN) * (16 * TJ);
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
  Acc acc[TI][TJ];
  double acc64[kMixed ? TI : 1][TJ][4];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      acc[i][j] = Acc{0, 0, 0, 0};
      if constexpr (kMixed) {
#pragma unroll
        for (int r = 0; r < 4; ++r) acc64[i][j][r] = 0.0;
      }
    }

  T va[TileA::E], vb[TileB::E];
  int buf = 0;
  constexpr int kCarrySlabs = kMixed ? (BK < 128 ? 128 / BK : 1) : 1;
  int ncarry = 0;
  if (kbeg < kend) {
    TileA::template fetch<VEC>(A, lda, M, kend, m0, kbeg, tid, va);
    TileB::template fetch<VEC>(B, ldb, N, kend, n0, kbeg, tid, vb);
    TileA::stash(As[0], tid, va);
    TileB::stash(Bs[0], tid, vb);
  }
  __syncthreads();
  const int row = lane & 15;
  const int kq = lane >> 4;
  for (int k0 = kbeg; k0 < kend; k0 += BK) {
    const bool more = k0 + BK < kend;
    if (more) {
      TileA::template fetch<VEC>(A, lda, M, kend, m0, k0 + BK, tid, va);
      TileB::template fetch<VEC>(B, ldb, N, kend, n0, k0 + BK, tid, vb);
    }
    const T* as = As[buf];
    const T* bs = Bs[buf];
#pragma unroll
    for (int kk = 0; kk < BK; kk += 4) {
      T av[TI], bv[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) av[i] = TileA::at(as, wm + i * 16 + row, kk + kq);
#pragma unroll
      for (int j = 0; j < TJ; ++j) bv[j] = TileB::at(bs, wn + j * 16 + row, kk + kq);
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) mma(acc[i][j], av[i], bv[j]);
    }
    if constexpr (kMixed) {
      // carry the fp32 partial sums of the last kCarrySlabs slabs in fp64
      if (++ncarry == kCarrySlabs || !more) {
        ncarry = 0;
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) {
#pragma unroll
            for (int r = 0; r < 4; ++r) acc64[i][j][r] += (double)acc[i][j][r];
            acc[i][j] = Acc{0, 0, 0, 0};
          }
      }
    }
    if (more) {
      TileA::stash(As[buf ^ 1], tid, va);
      TileB::stash(Bs[buf ^ 1], tid, vb);
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
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
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

template <typename T, typename Acc, typename TC, typename Gm, int Site, bool TA, bool TB>
void launch_kernel(bool vec, dim3 grid, hipStream_t st, const GemmArgs& g, const T* A, const T* B, TC* C,
                   int ksplit, long strideP, double* scratch) {
  if (vec)
    hipLaunchKernelGGL((gemm_nt_kernel<T, Acc, TC, Gm, true, TA, TB, Site>), grid, dim3(Gm::NT), 0, st, g.M, g.N, g.K,
                       g.alpha, A, g.lda, B, g.ldb, g.beta, C, g.ldc, g.strideA, g.strideB, g.strideC, g.zdiv, ksplit,
                       strideP, scratch);
  else
    hipLaunchKernelGGL((gemm_nt_kernel<T, Acc, TC, Gm, false, TA, TB, Site>), grid, dim3(Gm::NT), 0, st, g.M, g.N,
                       g.K, g.alpha, A, g.lda, B, g.ldb, g.beta, C, g.ldc, g.strideA, g.strideB, g.strideC, g.zdiv,
                       ksplit, strideP, scratch);
}

// AllowT: instantiate the K-major operand variants (general contractions only)
template <typename T, typename Acc, typename TC, typename Gm, int Site = 0, bool AllowT = false>
hipError_t launch_geo(const GemmArgs& g, const T* A, const T* B, TC* C, hipStream_t st, double* scratch,
                      size_t scratch_elems) {
  constexpr int BM = Gm::BM, BN = Gm::BN;
  if ((g.ta || g.tb) && !AllowT) return hipErrorInvalidValue;
  const int tiles = ((g.M + BM - 1) / BM) * ((g.N + BN - 1) / BN);
  // Split K when there are few tiles, choosing the factor so the workgroups fill whole rounds
  // of the resident slots (256 CUs x 2 workgroups of these geometries): the smallest factor
  // reaching 95 % of the slots in every round, else the best one found.  Skinny tiles (one
  // side 16) stream their operand with little work per byte and may split further.
  int ksplit = 1;
  if (g.K > 0 && sizeof(TC) == sizeof(double)) {
    constexpr long kSlots = 512;
    constexpr int kMaxSplit = (BM == 16 || BN == 16) ? 512 : 64;
    const long base = (long)tiles * g.batch;
    auto fill = [&](long ks) {
      const long w = base * ks;
      return (double)w / (double)(((w + kSlots - 1) / kSlots) * kSlots);
    };
    if (base < 4 * kSlots) {
      double best = fill(1);
      for (int ks = 2; ks <= kMaxSplit; ++ks) {
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
  // 16-byte loads: the contiguous extent of each operand (K for row-major, M or N for
  // K-major) and its leading dimension are multiples of the vector width, bases aligned
  constexpr int VW = 16 / sizeof(T);
  const bool va = (g.ta ? g.M % VW == 0 : g.K % VW == 0) && g.lda % VW == 0 && g.strideA % VW == 0 &&
                  (uintptr_t)A % 16 == 0;
  const bool vb = (g.tb ? g.N % VW == 0 : g.K % VW == 0) && g.ldb % VW == 0 && g.strideB % VW == 0 &&
                  (uintptr_t)B % 16 == 0;
  const bool vec = va && vb;
  dim3 grid(tiles, 1, g.batch * ksplit);
  const long strideP = (long)g.M * g.N;
  if constexpr (AllowT) {
    if (g.ta && g.tb) launch_kernel<T, Acc, TC, Gm, Site, true, true>(vec, grid, st, g, A, B, C, ksplit, strideP, scratch);
    else if (g.ta) launch_kernel<T, Acc, TC, Gm, Site, true, false>(vec, grid, st, g, A, B, C, ksplit, strideP, scratch);
    else if (g.tb) launch_kernel<T, Acc, TC, Gm, Site, false, true>(vec, grid, st, g, A, B, C, ksplit, strideP, scratch);
    else launch_kernel<T, Acc, TC, Gm, Site, false, false>(vec, grid, st, g, A, B, C, ksplit, strideP, scratch);
  } else {
    launch_kernel<T, Acc, TC, Gm, Site, false, false>(vec, grid, st, g, A, B, C, ksplit, strideP, scratch);
  }
  if (ksplit > 1) {
    const long total = (long)g.batch * g.M * g.N;
    const int nb = (int)std::min<long>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(splitk_reduce<Site>, dim3(nb), dim3(256), 0, st, g.M, g.N, ksplit, g.batch, g.alpha,
                       g.beta, scratch, strideP, reinterpret_cast<double*>(C), g.ldc, g.strideC);
  }
  return hipGetLastError();
}

// measured on gfx950 (ring, ladder and square shapes): fp64 best with 128x128x16 tiles at two
// workgroups per CU (64x128 and 128x64 tiles at three were 1-7 % slower); fp32 with fp64 carry
// best with 64x128x32 tiles at up to three workgroups per CU (8-20 % over 128x128x32 at one)
using GeoF64 = Geo<128, 128, 16, 2, 2, 2>;
using GeoF32 = Geo<64, 128, 32, 2, 2, 2, 2, 4>;
// products with one side of at most 16 (full contractions down to a small active-index
// block): a 256 x 16 (16 x 256) tile, four waves along the long side, each 64 x 16
using GeoF64SkinnyN = Geo<256, 16, 16, 4, 1, 2, 4, 1, true>;
using GeoF64SkinnyM = Geo<16, 256, 16, 1, 4, 2, 1, 4, true>;

template <typename T, typename Acc, typename TC>
hipError_t launch(const GemmArgs& g, const T* A, const T* B, TC* C, hipStream_t st, double* scratch,
                  size_t scratch_elems) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return hipSuccess;
  if (g.K <= 0 && g.beta == 1.0) return hipSuccess;
  if (g.site == 1) {
    // the ladder's products: row-major operands, the default tile shape of their type
    if constexpr (sizeof(T) == 8) return launch_geo<T, Acc, TC, GeoF64, 1>(g, A, B, C, st, scratch, scratch_elems);
    else return launch_geo<T, Acc, TC, GeoF32, 1>(g, A, B, C, st, scratch, scratch_elems);
  }
  if constexpr (sizeof(T) == 8) {
    if (g.N <= 16 && g.M > 16) return launch_geo<T, Acc, TC, GeoF64SkinnyN, 0, true>(g, A, B, C, st, scratch, scratch_elems);
    if (g.M <= 16 && g.N > 16) return launch_geo<T, Acc, TC, GeoF64SkinnyM, 0, true>(g, A, B, C, st, scratch, scratch_elems);
    return launch_geo<T, Acc, TC, GeoF64, 0, true>(g, A, B, C, st, scratch, scratch_elems);
  }
  else return launch_geo<T, Acc, TC, GeoF32, 0, sizeof(TC) == 8>(g, A, B, C, st, scratch, scratch_elems);
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
