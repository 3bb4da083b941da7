// Bandwidth-bound kernels of the residual engine (gfx950).
//
//  * strided copy/accumulate between tensor views (index permutation of the
//    contraction operands, scatter-add of contraction results);
//  * pair symmetrization X[k,l,c,d] + X[l,k,d,c] (eq. spinfree-perm-sym);
//  * the flow-regularized Jacobi update with its step norm (eq. ric-update);
//  * deterministic two-pass reductions (energy dot products, norms);
//  * density-cumulant preparation (Section 2.1 and 2.3.2) and the reference energy.
#include <hip/hip_runtime.h>
#include <algorithm>
#include <cstdint>
#include "kernels.h"

namespace ric {

namespace {

constexpr int kThreads = 256;
constexpr int kRedBlocks = kReducePartials;  // blocks of the two-pass reductions, one partial sum each

inline int blocks_for(long n, int per = kThreads) {
  long b = (n + per - 1) / per;
  if (b > 1048576) b = 1048576;
  return (int)(b < 1 ? 1 : b);
}

// ---- strided views ------------------------------------------------------------------

// out[o(i)] = beta * out[o(i)] + alpha * in[s(i)] over the iteration space of `it`
// Idx: unsigned 32-bit index arithmetic when the space has fewer than 2^32 elements (its
// divisions are far cheaper than 64-bit ones), else 64-bit.
template <typename TO, typename TI, typename Idx>
__global__ void __launch_bounds__(kThreads)
strided_axpby(Iter it, double alpha, const TI* __restrict__ in, double beta, TO* __restrict__ out) {
  const long total = it.total;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    Idx rem = (Idx)t;
    long so = 0, si = 0;
#pragma unroll
    for (int d = kMaxDims - 1; d >= 0; --d) {
      if (d < it.nd) {
        const Idx e = (Idx)it.ext[d];
        const Idx x = rem % e;
        rem /= e;
        so += (long)x * it.so[d];
        si += (long)x * it.si[d];
      }
    }
    const double v = alpha * (double)in[si];
    out[so] = beta == 0.0 ? (TO)v : (TO)(beta * (double)out[so] + v);
  }
}

// The same map when the output's stride-1 dimension (da) and the input's (db) differ: a
// workgroup moves a 32 x 32 tile of (da, db) through LDS, reading rows that are contiguous in
// the input and writing rows that are contiguous in the output, for one index of the other
// dimensions at a time (grid.y strides over them; the loop bounds are uniform per workgroup).
constexpr int kTile = 32;

template <typename TO, typename TI>
__global__ void __launch_bounds__(256)
strided_tile(Iter it, int da, int db, double alpha, const TI* __restrict__ in, double beta, TO* __restrict__ out) {
  __shared__ double tile[kTile][kTile + 1];
  const long ea = it.ext[da], eb = it.ext[db];
  const long nta = (ea + kTile - 1) / kTile;
  const long a0 = (long)(blockIdx.x % nta) * kTile, b0 = (long)(blockIdx.x / nta) * kTile;
  const int tx = threadIdx.x & (kTile - 1), ty = threadIdx.x / kTile;
  const long sia = it.si[da], sob = it.so[db];
  long outer = 1;
  for (int d = 0; d < it.nd; ++d)
    if (d != da && d != db) outer *= it.ext[d];
  for (long o = blockIdx.y; o < outer; o += gridDim.y) {
    long rem = o, bi = 0, bo = 0;
    for (int d = it.nd - 1; d >= 0; --d) {
      if (d == da || d == db) continue;
      const long e = it.ext[d], x = rem % e;
      rem /= e;
      bi += x * it.si[d];
      bo += x * it.so[d];
    }
    for (int j = ty; j < kTile; j += 256 / kTile) {
      const long a = a0 + j, b = b0 + tx;
      if (a < ea && b < eb) tile[j][tx] = (double)in[bi + a * sia + b];
    }
    __syncthreads();
    for (int j = ty; j < kTile; j += 256 / kTile) {
      const long b = b0 + j, a = a0 + tx;
      if (a < ea && b < eb) {
        const long oo = bo + a + b * sob;
        const double v = alpha * tile[tx][j];
        out[oo] = beta == 0.0 ? (TO)v : (TO)(beta * (double)out[oo] + v);
      }
    }
    __syncthreads();
  }
}

__global__ void fill_kernel(double* __restrict__ p, long n, double v) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) p[t] = v;
}

// X[k,l,c,d] <- scale (X[k,l,c,d] + X[l,k,d,c]) over [nh][nh][np][np].  One workgroup takes a
// hole pair k <= l (grid.y) and a 32 x 32 tile (C, D) of the particle pairs (grid.x): it reads
// the tile of the (k, l) matrix and the mirrored tile (D, C) of the (l, k) matrix with
// row-contiguous loads, transposes the mirror through LDS, and writes the symmetrized values
// to both places.  For k == l only the tiles C <= D run (they cover the mirror as well).
constexpr int kSymTile = 32;

__global__ void __launch_bounds__(256) symmetrize_kernel(double* __restrict__ x, int nh, int np, double scale) {
  constexpr int TS = kSymTile;
  __shared__ double a[TS][TS + 1];
  __shared__ double b[TS][TS + 1];
  const int nt = (np + TS - 1) / TS;
  const int CB = blockIdx.x / nt, DB = blockIdx.x % nt;
  const long pairs = (long)nh * (nh + 1) / 2;
  const long pp = (long)np * np;
  // hole pairs k <= l by the packed index pr = l (l + 1) / 2 + k; the loop bounds and the skip
  // are uniform over the workgroup, so its barriers are reached by every thread
  for (long pr = blockIdx.y; pr < pairs; pr += gridDim.y) {
  int l = (int)((sqrt(8.0 * pr + 1.0) - 1.0) / 2.0);
  while ((long)l * (l + 1) / 2 > pr) --l;
  while ((long)(l + 1) * (l + 2) / 2 <= pr) ++l;
  const int k = (int)(pr - (long)l * (l + 1) / 2);
  if (k == l && CB > DB) continue;
  double* xkl = x + ((long)k * nh + l) * pp;
  double* xlk = x + ((long)l * nh + k) * pp;
  const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
  constexpr int RPP = 256 / TS;
  for (int i = ty; i < TS; i += RPP) {
    const int c = CB * TS + i, d = DB * TS + tx;
    a[i][tx] = (c < np && d < np) ? xkl[(long)c * np + d] : 0.0;       // X[k,l,c,d]
    const int d2 = DB * TS + i, c2 = CB * TS + tx;
    b[i][tx] = (d2 < np && c2 < np) ? xlk[(long)d2 * np + c2] : 0.0;    // X[l,k,d2,c2]
  }
  __syncthreads();
  for (int i = ty; i < TS; i += RPP) {
    const int c = CB * TS + i, d = DB * TS + tx;
    if (c < np && d < np) xkl[(long)c * np + d] = scale * (a[i][tx] + b[tx][i]);
    const int d2 = DB * TS + i, c2 = CB * TS + tx;
    if (d2 < np && c2 < np) xlk[(long)d2 * np + c2] = scale * (b[i][tx] + a[tx][i]);
  }
  __syncthreads();   // the next pair overwrites the tiles
  }
}

// zero the amplitude blocks whose indices are all active (Section 2.2)
__global__ void mask_kernel(double* __restrict__ r1, double* __restrict__ r2, int nc, int na, int nh, int np) {
  const long n2 = (long)na * na * na * na;
  const long n1 = (long)na * na;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n2 + n1; t += (long)gridDim.x * blockDim.x) {
    if (t < n2) {
      const int d = (int)(t % na), c = (int)((t / na) % na);
      const int l = (int)((t / n1) % na), k = (int)(t / (n1 * na));
      r2[(((long)(nc + k) * nh + nc + l) * np + c) * np + d] = 0.0;
    } else if (r1 != nullptr) {
      const long s = t - n2;
      const int c = (int)(s % na), k = (int)(s / na);
      r1[(long)(nc + k) * np + c] = 0.0;
    }
  }
}

// ---- reductions ------------------------------------------------------------------------

__device__ inline double block_sum(double v) {
  __shared__ double sh[kThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    for (int i = 0; i < kThreads / 64; ++i) s += sh[i];
  }
  __syncthreads();
  return s;
}

// partial[b] = sum over the b-th contiguous share of a[i]*b[i]
__global__ void __launch_bounds__(kThreads) dot_partial(const double* __restrict__ a, const double* __restrict__ b,
                                                        long n, double* __restrict__ partial) {
  const long per = (n + gridDim.x - 1) / gridDim.x;
  const long beg = blockIdx.x * per;
  const long end = beg + per < n ? beg + per : n;
  double s = 0.0;
  for (long i = beg + threadIdx.x; i < end; i += blockDim.x) s += a[i] * b[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// out[0] (+)= alpha * sum(partial[0..n))  in a fixed order
__global__ void finish_sum(const double* __restrict__ partial, int n, double alpha, double* __restrict__ out,
                           int accumulate) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) s += partial[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[0] = accumulate ? out[0] + alpha * s : alpha * s;
}

// ---- regularized update -------------------------------------------------------------------

// (k, l, c, d) of element u of a [nh][nh][np][np] array; 32-bit divisions below 2^32 elements
__device__ inline void amp2_index(long u, int nh, int np, int& k, int& l, int& c, int& d) {
  if (u < 4294967296L) {
    unsigned v = (unsigned)u;
    d = (int)(v % (unsigned)np);
    v /= (unsigned)np;
    c = (int)(v % (unsigned)np);
    v /= (unsigned)np;
    l = (int)(v % (unsigned)nh);
    k = (int)(v / (unsigned)nh);
  } else {
    d = (int)(u % np);
    c = (int)((u / np) % np);
    l = (int)((u / ((long)np * np)) % nh);
    k = (int)(u / ((long)np * np * nh));
  }
}

__device__ inline double phi(double D, double s) {
  // (1 - exp(-s D^2)) / D with the limit 0 at D = 0
  if (D == 0.0) return 0.0;
  return -expm1(-s * D * D) / D;
}

// Position of a wave's lane in the flat [nh][nh][np][np] doubles array: the element's
// particle index d and its row (k, l, c) with the row's hole part of Delta and its mask.
struct Amp2Cursor {
  int k, l, c, d;
  double dh;
  bool mrow;
};

__device__ inline void cursor_row(Amp2Cursor& q, const double* eps, const double* epsP, int nc, int na) {
  q.dh = eps[q.k] + eps[q.l] - epsP[q.c];
  q.mrow = q.k >= nc && q.l >= nc && q.c < na;   // T2 all-active left out (with d < na)
}

// Step the cursor by `by` elements along the flat array (rows advance in (k, l, c) order).
__device__ inline void cursor_step(Amp2Cursor& q, int by, int nh, int np, const double* eps, const double* epsP,
                                   int nc, int na) {
  q.d += by;
  if (q.d < np) return;
  while (q.d >= np) {
    q.d -= np;
    if (++q.c == np) {
      q.c = 0;
      if (++q.l == nh) {
        q.l = 0;
        ++q.k;
      }
    }
  }
  if (q.k < nh) cursor_row(q, eps, epsP, nc, na);
}

// The regularized update over T1 and T2 with each block's share of sum (t_new - t)^2.
// T2 is read as one flat stream: each wave takes a contiguous span of it, its 64 lanes on
// consecutive elements, four elements per lane in flight; a lane's row indices and Delta
// follow it incrementally, with no division per element.
__global__ void __launch_bounds__(kThreads)
update_kernel(double* __restrict__ t1, double* __restrict__ t2, const double* __restrict__ r1,
              const double* __restrict__ r2, const double* __restrict__ eps, int nc, int na, int nv,
              double s, double* __restrict__ partial) {
  const int nh = nc + na, np = na + nv;
  const double* epsP = eps + nc;
  double acc = 0.0;
  const long n1 = (long)nh * np;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n1; i += (long)gridDim.x * blockDim.x) {
    const int k = (int)(i / np), d = (int)(i - (long)k * np);
    if (k >= nc && d < na) continue;      // T1 active -> active left out
    const double D = eps[k] - epsP[d];
    const double tv = t1[i];
    const double nw = (tv * D + r1[i]) * phi(D, s);
    const double dv = nw - tv;
    acc += dv * dv;
    t1[i] = nw;
  }
  constexpr int kU = 4;                    // elements per lane in flight
  const long n2 = n1 * n1;
  const int lane = threadIdx.x & 63;
  const long waves = (long)gridDim.x * (blockDim.x >> 6);
  const long wid = (long)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const long span = ((n2 + waves - 1) / waves + 64 * kU - 1) / (64 * kU) * (64 * kU);
  const long beg = wid * span, end = beg + span < n2 ? beg + span : n2;
  if (beg + lane < end) {
    Amp2Cursor q;
    amp2_index(beg + lane, nh, np, q.k, q.l, q.c, q.d);
    cursor_row(q, eps, epsP, nc, na);
    for (long i = beg + lane; i < end; i += 64 * kU) {
      long idx[kU];
      double D[kU], tv[kU], rv[kU];
      bool on[kU];
#pragma unroll
      for (int j = 0; j < kU; ++j) {
        idx[j] = i + 64L * j;
        on[j] = idx[j] < end && !(q.mrow && q.d < na);
        D[j] = q.dh - epsP[q.d < np ? q.d : 0];
        if (j + 1 < kU) cursor_step(q, 64, nh, np, eps, epsP, nc, na);
      }
#pragma unroll
      for (int j = 0; j < kU; ++j) {
        tv[j] = on[j] ? t2[idx[j]] : 0.0;
        rv[j] = on[j] ? r2[idx[j]] : 0.0;
      }
#pragma unroll
      for (int j = 0; j < kU; ++j) {
        if (!on[j]) continue;
        const double nw = (tv[j] * D[j] + rv[j]) * phi(D[j], s);
        const double dv = nw - tv[j];
        acc += dv * dv;
        t2[idx[j]] = nw;
      }
      cursor_step(q, 64, nh, np, eps, epsP, nc, na);
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// d phi / d D, with the series s (1 - 3/2 x + 5/6 x^2), x = s D^2, where the closed form cancels
__device__ inline double dphi(double D, double s) {
  const double x = s * D * D;
  if (x < 1e-4) return s * (1.0 - 1.5 * x + (5.0 / 6.0) * x * x);
  const double e = exp(-x);
  return (2.0 * x * e + expm1(-x)) / (D * D);
}

// Lagrangian iteration L <- g + Delta phi L + j over the stored amplitudes (the excluded
// all-active blocks stay zero); partial[b] = sum over the block's share of (L_new - L)^2
__global__ void __launch_bounds__(kThreads)
lambda_kernel(double* __restrict__ l1, double* __restrict__ l2, const double* __restrict__ g1,
              const double* __restrict__ g2, const double* __restrict__ j1, const double* __restrict__ j2,
              const double* __restrict__ eps, int nc, int na, int nv, double s, double* __restrict__ partial) {
  const int nh = nc + na, np = na + nv;
  const long n1 = (long)nh * np;
  const long total = n1 + (long)nh * nh * np * np;
  const long per = (total + gridDim.x - 1) / gridDim.x;
  const long beg = blockIdx.x * per;
  const long end = beg + per < total ? beg + per : total;
  double acc = 0.0;
  for (long t = beg + threadIdx.x; t < end; t += blockDim.x) {
    double* l;
    double g, j, D;
    bool masked;
    if (t < n1) {
      const int k = (int)(t / np), c = (int)(t % np);
      masked = k >= nc && c < na;
      D = eps[k] - eps[nc + c];
      l = l1 + t;
      g = g1[t];
      j = j1[t];
    } else {
      const long u = t - n1;
      int k, ll, c, d;
      amp2_index(u, nh, np, k, ll, c, d);
      masked = k >= nc && ll >= nc && c < na && d < na;
      D = eps[k] + eps[ll] - eps[nc + c] - eps[nc + d];
      l = l2 + u;
      g = g2[u];
      j = j2[u];
    }
    const double nw = masked ? 0.0 : g + D * phi(D, s) * l[0] + j;
    const double dv = nw - l[0];
    acc += dv * dv;
    l[0] = nw;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// out = phi(Delta) * L, zero on the excluded blocks
__global__ void flow_scale_kernel(const double* __restrict__ l1, const double* __restrict__ l2,
                                  const double* __restrict__ eps, int nc, int na, int nv, double s,
                                  double* __restrict__ o1, double* __restrict__ o2) {
  const int nh = nc + na, np = na + nv;
  const long n1 = (long)nh * np;
  const long total = n1 + (long)nh * nh * np * np;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    if (t < n1) {
      const int k = (int)(t / np), c = (int)(t % np);
      const double D = eps[k] - eps[nc + c];
      o1[t] = (k >= nc && c < na) ? 0.0 : phi(D, s) * l1[t];
    } else {
      const long u = t - n1;
      int k, ll, c, d;
      amp2_index(u, nh, np, k, ll, c, d);
      const double D = eps[k] + eps[ll] - eps[nc + c] - eps[nc + d];
      o2[u] = (k >= nc && ll >= nc && c < na && d < na) ? 0.0 : phi(D, s) * l2[u];
    }
  }
}

// w = L [T phi + (T Delta + R) phi'] of one amplitude (its dU/dDelta weighted by L)
__device__ inline double flow_weight(double l, double t, double r, double D, double s) {
  return l * (t * phi(D, s) + (t * D + r) * dphi(D, s));
}

// dF[p,p] += sum over amplitudes of w * dDelta/df_pp: +1 per hole index equal to p, -1 per
// particle index equal to p.  One workgroup per orbital p, summed in a fixed order.
__global__ void __launch_bounds__(kThreads)
flow_fock_kernel(const double* __restrict__ t1, const double* __restrict__ t2, const double* __restrict__ r1,
                 const double* __restrict__ r2, const double* __restrict__ l1, const double* __restrict__ l2,
                 const double* __restrict__ eps, int nc, int na, int nv, double s, double* __restrict__ df) {
  const int nh = nc + na, np = na + nv, n = nc + na + nv;
  const int p = blockIdx.x;
  const long pp = (long)np * np;
  double acc = 0.0;
  auto w1 = [&](int k, int c) {
    if (k >= nc && c < na) return 0.0;
    const long i = (long)k * np + c;
    return flow_weight(l1[i], t1[i], r1[i], eps[k] - eps[nc + c], s);
  };
  auto w2 = [&](int k, int l, int c, int d) {
    if (k >= nc && l >= nc && c < na && d < na) return 0.0;
    const long i = (((long)k * nh + l) * np + c) * np + d;
    return flow_weight(l2[i], t2[i], r2[i], eps[k] + eps[l] - eps[nc + c] - eps[nc + d], s);
  };
  if (p < nh) {
    for (long i = threadIdx.x; i < np; i += blockDim.x) acc += w1(p, (int)i);
    for (long i = threadIdx.x; i < (long)nh * pp; i += blockDim.x) {
      const int l = (int)(i / pp), c = (int)((i / np) % np), d = (int)(i % np);
      acc += w2(p, l, c, d) + w2(l, p, c, d);
    }
  }
  if (p >= nc) {
    const int c = p - nc;
    for (long i = threadIdx.x; i < nh; i += blockDim.x) acc -= w1((int)i, c);
    for (long i = threadIdx.x; i < (long)nh * nh * np; i += blockDim.x) {
      const int k = (int)(i / ((long)nh * np)), l = (int)((i / np) % nh), e = (int)(i % np);
      acc -= w2(k, l, c, e) + w2(k, l, e, c);
    }
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) df[(long)p * n + p] += acc;
}

// ---- generalized Fock matrix from h (Section 2.1) --------------------------------------------

// w[p,q] = 2 delta_pq on core orbitals, Gamma1[t,u] on the active block, 0 elsewhere: the
// spin-summed 1-RDM of the reference
__global__ void fock_weights_kernel(double* __restrict__ w, int n, int nc, int na, const double* __restrict__ g1) {
  const long total = (long)n * n;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const int p = (int)(t / n), q = (int)(t % n);
    double v = 0.0;
    if (p < nc && q < nc) v = p == q ? 2.0 : 0.0;
    else if (p >= nc && p < nc + na && q >= nc && q < nc + na) v = g1[(p - nc) * na + (q - nc)];
    w[t] = v;
  }
}

// out[i] += alpha * sum_X B[X][i] d[X] over the n2 columns i of B (row-major [nx][n2])
__global__ void column_dot_kernel(const double* __restrict__ B, const double* __restrict__ d, int nx, long n2,
                                  double alpha, double* __restrict__ out) {
  for (long i = blockIdx.x * (long)blockDim.x + threadIdx.x; i < n2; i += (long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int x = 0; x < nx; ++x) s += B[(long)x * n2 + i] * d[x];
    out[i] += alpha * s;
  }
}

// Column j of the m x m block at u (row stride ld): flip its sign unless its entry of largest
// magnitude (the first one on ties) is positive.  One workgroup per column.
__global__ void __launch_bounds__(kThreads) column_sign_kernel(double* __restrict__ u, int m, long ld) {
  __shared__ double bv[kThreads];
  __shared__ int bi[kThreads];
  const int j = blockIdx.x;
  double best = -1.0;
  int arg = m;
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const double a = fabs(u[(long)i * ld + j]);
    if (a > best) {
      best = a;
      arg = i;
    }
  }
  bv[threadIdx.x] = best;
  bi[threadIdx.x] = arg;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      const double o = bv[threadIdx.x + w];
      const int oi = bi[threadIdx.x + w];
      if (o > bv[threadIdx.x] || (o == bv[threadIdx.x] && oi < bi[threadIdx.x])) {
        bv[threadIdx.x] = o;
        bi[threadIdx.x] = oi;
      }
    }
    __syncthreads();
  }
  const int piv = bi[0];
  const bool flip = piv < m && u[(long)piv * ld + j] < 0.0;
  __syncthreads();
  if (flip)
    for (int i = threadIdx.x; i < m; i += blockDim.x) u[(long)i * ld + j] = -u[(long)i * ld + j];
}

__global__ void diag_kernel(const double* __restrict__ f, int n, double* __restrict__ eps) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) eps[i] = f[(long)i * n + i];
}

__global__ void nonfinite_kernel(const double* __restrict__ x, long n, int* __restrict__ flag) {
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x)
    if (!isfinite(x[t])) flag[0] = 1;
}

// ---- density cumulants (Section 2.1, 2.3.2) ------------------------------------------------

// gA = Gamma1 / 2 (per-spin 1-RDM), eA = 1 - Gamma1 / 2 (per-spin 1-hole RDM)
__global__ void onebody_kernel(const double* __restrict__ g1, int na, double* __restrict__ ga, double* __restrict__ ea) {
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < na * na; t += gridDim.x * blockDim.x) {
    const double h = 0.5 * g1[t];
    ga[t] = h;
    ea[t] = ((t / na) == (t % na) ? 1.0 : 0.0) - h;
  }
}

// Lambda2[p,q,r,s] = G2 - G1[p,r] G1[q,s] + 1/2 G1[p,s] G1[q,r]
__global__ void lambda2_kernel(const double* __restrict__ g1, const double* __restrict__ g2, int na,
                               double* __restrict__ l2) {
  const long n = (long)na * na * na * na;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const int s = (int)(t % na), r = (int)((t / na) % na), q = (int)((t / ((long)na * na)) % na),
              p = (int)(t / ((long)na * na * na));
    l2[t] = g2[t] - g1[p * na + r] * g1[q * na + s] + 0.5 * g1[p * na + s] * g1[q * na + r];
  }
}

// K2[p,q,r,s] = (2 Lambda2[p,q,r,s] + Lambda2[p,q,s,r]) / 6: kernel of the two-delta spin
// expansion of the two-body cumulant
__global__ void k2_kernel(const double* __restrict__ l2, int na, double* __restrict__ k2) {
  const long n = (long)na * na * na * na;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    const int s = (int)(t % na), r = (int)((t / na) % na);
    const long base = t - (long)r * na - s;
    k2[t] = (2.0 * l2[t] + l2[base + (long)s * na + r]) / 6.0;
  }
}

__device__ inline long ix6(int na, int a, int b, int c, int d, int e, int f) {
  return ((((((long)a * na + b) * na + c) * na + d) * na + e) * na + f);
}
__device__ inline long ix4(int na, int a, int b, int c, int d) {
  return ((((long)a * na + b) * na + c) * na + d);
}

// Lambda3 (spin-free three-body cumulant of a singlet) from Gamma3, Gamma1 and Lambda2
__global__ void lambda3_kernel(const double* __restrict__ G, const double* __restrict__ L,
                               const double* __restrict__ g3, int na, double* __restrict__ l3) {
  const long n = (long)na * na * na * na * na * na;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    long r0 = t;
    const int u = (int)(r0 % na); r0 /= na;
    const int tt = (int)(r0 % na); r0 /= na;
    const int s = (int)(r0 % na); r0 /= na;
    const int r = (int)(r0 % na); r0 /= na;
    const int q = (int)(r0 % na); r0 /= na;
    const int p = (int)r0;
#define G1(a, b) G[(a) * na + (b)]
#define L2(a, b, c, d) L[ix4(na, a, b, c, d)]
    double v = g3[t];
    v -= G1(p, s) * L2(q, r, tt, u) + G1(q, tt) * L2(p, r, s, u) + G1(r, u) * L2(p, q, s, tt);
    v += 0.5 * (G1(p, tt) * L2(q, r, s, u) + G1(p, u) * L2(q, r, tt, s) + G1(q, s) * L2(p, r, tt, u) +
                G1(q, u) * L2(p, r, s, tt) + G1(r, s) * L2(p, q, u, tt) + G1(r, tt) * L2(p, q, s, u));
    v -= G1(p, s) * G1(q, tt) * G1(r, u);
    v += 0.5 * (G1(p, s) * G1(q, u) * G1(r, tt) + G1(p, tt) * G1(q, s) * G1(r, u) + G1(p, u) * G1(q, tt) * G1(r, s));
    v -= 0.25 * (G1(p, tt) * G1(q, u) * G1(r, s) + G1(p, u) * G1(q, s) * G1(r, tt));
#undef G1
#undef L2
    l3[t] = v;
  }
}

// K3[pqr;stu] = sum_pi w_pi Lambda3[pqr; pi(stu)], w = 17/144 (identity), -1/144
// (transpositions), -7/144 (three-cycles): kernel of the spin-delta expansion of lambda3
__global__ void k3_kernel(const double* __restrict__ l3, int na, double* __restrict__ k3) {
  const long n = (long)na * na * na * na * na * na;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < n; t += (long)gridDim.x * blockDim.x) {
    long r0 = t;
    const int u = (int)(r0 % na); r0 /= na;
    const int tt = (int)(r0 % na); r0 /= na;
    const int s = (int)(r0 % na); r0 /= na;
    const int r = (int)(r0 % na); r0 /= na;
    const int q = (int)(r0 % na); r0 /= na;
    const int p = (int)r0;
    const double v = 17.0 * l3[t] - l3[ix6(na, p, q, r, tt, s, u)] - l3[ix6(na, p, q, r, u, tt, s)] -
                     l3[ix6(na, p, q, r, s, u, tt)] - 7.0 * l3[ix6(na, p, q, r, tt, u, s)] -
                     7.0 * l3[ix6(na, p, q, r, u, s, tt)];
    k3[t] = v / 144.0;
  }
}

// Reference energy from f, the (hh|hh) integral block and the active RDMs:
// E0 = 2 sum_i f_ii + sum_tu f_tu G_tu - 2 sum_ij (ii|jj) + sum_ij (ij|ji)
//      - 2 sum_i,tu (ii|tu) G_tu + sum_i,tu (iu|ti) G_tu - sum G_tu G_vw (tu|vw)
//      + 1/2 sum G_tu G_vw (tw|vu) + 1/2 sum (tv|uw) G2[t,u,v,w]
__global__ void e0_kernel(const double* __restrict__ f, int n, const double* __restrict__ I4, int nc, int na,
                          const double* __restrict__ g1, const double* __restrict__ g2, double* __restrict__ out) {
  const int nh = nc + na;
  auto eri = [&](int p, int r, int q, int s) { return I4[(((long)p * nh + r) * nh + q) * nh + s]; };
  double acc = 0.0;
  for (int i = threadIdx.x; i < nc; i += blockDim.x) acc += 2.0 * f[(long)i * n + i];
  for (int x = threadIdx.x; x < na * na; x += blockDim.x) {
    const int t = x / na, u = x % na;
    acc += f[(long)(nc + t) * n + nc + u] * g1[x];
  }
  for (int x = threadIdx.x; x < nc * nc; x += blockDim.x) {
    const int i = x / nc, j = x % nc;
    acc += -2.0 * eri(i, i, j, j) + eri(i, j, j, i);
  }
  for (long x = threadIdx.x; x < (long)nc * na * na; x += blockDim.x) {
    const int i = (int)(x / (na * na)), t = (int)((x / na) % na), u = (int)(x % na);
    const double g = g1[t * na + u];
    acc += -2.0 * eri(i, i, nc + t, nc + u) * g + eri(i, nc + u, nc + t, i) * g;
  }
  const long na4 = (long)na * na * na * na;
  for (long x = threadIdx.x; x < na4; x += blockDim.x) {
    const int w = (int)(x % na), v = (int)((x / na) % na), u = (int)((x / ((long)na * na)) % na),
              t = (int)(x / ((long)na * na * na));
    const double gtu = g1[t * na + u], gvw = g1[v * na + w];
    acc += -gtu * gvw * eri(nc + t, nc + u, nc + v, nc + w) + 0.5 * gtu * gvw * eri(nc + t, nc + w, nc + v, nc + u);
    acc += 0.5 * eri(nc + t, nc + v, nc + u, nc + w) * g2[x];
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) out[0] = acc;
}

// ladder scatter: C[kl][(c - c0) * ncol + d] -> R2[k,l,c,d] and, for d < c, R2[l,k,d,c]
__global__ void ladder_scatter(const double* __restrict__ Cm, int nh, int np, int c0, int c1, int ncol,
                               double* __restrict__ r2) {
  const long rows = (long)nh * nh;
  const long cols = (long)(c1 - c0) * ncol;
  const long total = rows * cols;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long kl = t / cols;
    const long j = t % cols;
    const int c = c0 + (int)(j / ncol);
    const int d = (int)(j % ncol);
    if (d > c) continue;
    const int k = (int)(kl / nh), l = (int)(kl % nh);
    if (d == c && k > l) continue;  // (l,k,c,c) is written from (k,l,c,c) so R2 stays exactly pair-symmetric
    const double v = Cm[t];
    r2[(((long)k * nh + l) * np + c) * np + d] += v;
    if (d < c || k < l) r2[(((long)l * nh + k) * np + d) * np + c] += v;
  }
}

// ---- pair-packed ladder (+/- combinations) -----------------------------------------------
// Packed pair index of (e, f) with e >= f: e (e + 1) / 2 + f; strict e > f: e (e - 1) / 2 + f.

// tau+[kl][ef] = w (tau[k,l,e,f] + tau[k,l,f,e]) / 2 for k <= l, e >= f (w = 1/2 on e == f)
// tau-[kl][ef] = (tau[k,l,e,f] - tau[k,l,f,e]) / 2       for k <  l, e >  f
template <typename TO>
__global__ void pack_tau_kernel(const double* __restrict__ tau, int nh, int np, TO* __restrict__ tp,
                                TO* __restrict__ tm, long ldp, long ldm) {
  const long nhp = (long)nh * (nh + 1) / 2, npp = (long)np * (np + 1) / 2;
  const long nhm = (long)nh * (nh - 1) / 2, npm = (long)np * (np - 1) / 2;
  const long total = nhp * ldp + nhm * ldm;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const bool plus = t < nhp * ldp;
    const long u = plus ? t : t - nhp * ldp;
    const long ld = plus ? ldp : ldm;
    const long r = u / ld, q = u % ld;
    if (q >= (plus ? npp : npm)) {  // zero padding of the packed rows
      if (plus) tp[u] = (TO)0; else tm[u] = (TO)0;
      continue;
    }
    // row r -> (k, l), k <= l (plus) or k < l (minus), enumerated by l
    int l = (int)((sqrt(8.0 * r + 1.0) - 1.0) / 2.0);
    if (plus) {
      while ((long)l * (l + 1) / 2 > r) --l;
      while ((long)(l + 1) * (l + 2) / 2 <= r) ++l;
    } else {
      l = (int)((sqrt(8.0 * r + 1.0) + 1.0) / 2.0);
      while ((long)l * (l - 1) / 2 > r) --l;
      while ((long)(l + 1) * l / 2 <= r) ++l;
    }
    const int k = plus ? (int)(r - (long)l * (l + 1) / 2) : (int)(r - (long)l * (l - 1) / 2);
    int e;
    if (plus) {
      e = (int)((sqrt(8.0 * q + 1.0) - 1.0) / 2.0);
      while ((long)e * (e + 1) / 2 > q) --e;
      while ((long)(e + 1) * (e + 2) / 2 <= q) ++e;
    } else {
      e = (int)((sqrt(8.0 * q + 1.0) + 1.0) / 2.0);
      while ((long)e * (e - 1) / 2 > q) --e;
      while ((long)(e + 1) * e / 2 <= q) ++e;
    }
    const int f = plus ? (int)(q - (long)e * (e + 1) / 2) : (int)(q - (long)e * (e - 1) / 2);
    const long base = ((long)k * nh + l) * np;
    const double a = tau[(base + e) * np + f];
    const double b = tau[(base + f) * np + e];
    if (plus) tp[u] = (TO)((e == f ? 0.25 : 0.5) * (a + b));
    else tm[u] = (TO)(0.5 * (a - b));
  }
}

// W+[(c,d)][ef] = W'[c][e][d][f] + W'[c][f][d][e] (e >= f), W-[(c,d)][ef] = difference (e > f),
// for c in [c0, c1), d < c1; W' rows (c, e) of length c1 * np.  For one pair (c, d) the
// np x np matrix M[e][f] = W'[c][e][d][f] is read as 32 x 32 tiles: a workgroup loads the
// tile (E, F), E >= F, and its mirror (F, E) with row-contiguous reads into LDS, so that
// M[f][e] comes from LDS instead of a column walk through HBM, and writes the packed
// triangles row by row.  grid.x: tile pairs, grid.y: (c, d) pairs.
constexpr int kPackTile = 32;

template <typename T>
__global__ void __launch_bounds__(256) pack_w_kernel(const T* __restrict__ wsrc, int np, long pairs, int c1,
                                                     T* __restrict__ wp, T* __restrict__ wm, long ldp, long ldm) {
  constexpr int TS = kPackTile;
  __shared__ T tile[2][TS][TS + 1];
  const long npp = (long)np * (np + 1) / 2, npm = (long)np * (np - 1) / 2;
  const int tp = blockIdx.x;
  int E = (int)((sqrt(8.0 * tp + 1.0) - 1.0) / 2.0);
  while (E * (E + 1) / 2 > tp) --E;
  while ((E + 1) * (E + 2) / 2 <= tp) ++E;
  const int F = tp - E * (E + 1) / 2;
  const long ld = (long)c1 * np;
  const int tx = threadIdx.x % TS, ty = threadIdx.x / TS;
  constexpr int kRowsPerPass = 256 / TS;
  for (long pr = blockIdx.y; pr < pairs; pr += gridDim.y) {   // block-uniform: the barriers below are safe
  const int cr = (int)(pr / c1), d = (int)(pr % c1);
  const T* base = wsrc + (long)cr * np * ld + (long)d * np;   // M[e][f] = base[e * ld + f]
  for (int i = ty; i < TS; i += kRowsPerPass) {
    const int e = E * TS + i, f = F * TS + tx;
    tile[0][i][tx] = (e < np && f < np) ? base[(long)e * ld + f] : (T)0;        // M[E*TS+i][F*TS+tx]
    const int e2 = F * TS + i, f2 = E * TS + tx;
    tile[1][i][tx] = (e2 < np && f2 < np) ? base[(long)e2 * ld + f2] : (T)0;    // M[F*TS+i][E*TS+tx]
  }
  __syncthreads();
  for (int i = ty; i < TS; i += kRowsPerPass) {
    const int e = E * TS + i, f = F * TS + tx;
    if (e >= np || f > e) continue;
    const T a = tile[0][i][tx];    // M[e][f]
    const T b = tile[1][tx][i];    // M[f][e]
    wp[pr * ldp + (long)e * (e + 1) / 2 + f] = a + b;
    if (f < e) wm[pr * ldm + (long)e * (e - 1) / 2 + f] = a - b;
  }
  if (tp == 0) {
    for (long q = npp + threadIdx.x; q < ldp; q += blockDim.x) wp[pr * ldp + q] = (T)0;
    for (long q = npm + threadIdx.x; q < ldm; q += blockDim.x) wm[pr * ldm + q] = (T)0;
  }
  __syncthreads();   // the next pair overwrites the tiles
  }
}

// R2 from S+[kl+][(c - c0) c1 + d] and S-[kl-][...] for d <= c (pair symmetry fills d > c)
__global__ void ladder_scatter_pm(const double* __restrict__ sp, const double* __restrict__ sm, int nh, int np,
                                  int c0, int c1, double* __restrict__ r2) {
  const long nhp = (long)nh * (nh + 1) / 2;
  const long cols = (long)(c1 - c0) * c1;
  const long total = nhp * cols;
  for (long t = blockIdx.x * (long)blockDim.x + threadIdx.x; t < total; t += (long)gridDim.x * blockDim.x) {
    const long r = t / cols, j = t % cols;
    const int c = c0 + (int)(j / c1), d = (int)(j % c1);
    if (d > c) continue;
    int l = (int)((sqrt(8.0 * r + 1.0) - 1.0) / 2.0);
    while ((long)l * (l + 1) / 2 > r) --l;
    while ((long)(l + 1) * (l + 2) / 2 <= r) ++l;
    const int k = (int)(r - (long)l * (l + 1) / 2);
    const double vp = sp[t];
    // the minus part vanishes identically for k == l and for c == d
    const double vm = (k < l && d < c) ? sm[((long)l * (l - 1) / 2 + k) * cols + j] : 0.0;
    const double a = vp + vm, b = vp - vm;   // (k,l,c,d) and (l,k,c,d)
    r2[(((long)k * nh + l) * np + c) * np + d] += a;
    if (k < l) r2[(((long)l * nh + k) * np + c) * np + d] += b;
    if (d < c) {
      r2[(((long)l * nh + k) * np + d) * np + c] += a;
      if (k < l) r2[(((long)k * nh + l) * np + d) * np + c] += b;
    }
  }
}

}  // namespace

// ---- launchers ------------------------------------------------------------------------------

template <typename TO, typename TI>
hipError_t launch_strided(const Iter& it, double alpha, const TI* in, double beta, TO* out, hipStream_t st) {
  if (it.total <= 0) return hipSuccess;
  // a transposing map (the stride-1 dimensions of output and input differ) of some size goes
  // through LDS tiles; the element-wise kernel reads such an input a stride apart
  int da = -1, db = -1;
  for (int d = 0; d < it.nd; ++d) {
    if (da < 0 && it.so[d] == 1 && it.ext[d] > 1) da = d;
    if (db < 0 && it.si[d] == 1 && it.ext[d] > 1) db = d;
  }
  if (da >= 0 && db >= 0 && da != db && it.ext[da] >= 16 && it.ext[db] >= 16 && it.total >= (1L << 16)) {
    const long nt = ((it.ext[da] + kTile - 1) / kTile) * ((it.ext[db] + kTile - 1) / kTile);
    const long outer = it.total / (it.ext[da] * it.ext[db]);
    if (nt < (1L << 31)) {
      hipLaunchKernelGGL((strided_tile<TO, TI>), dim3((unsigned)nt, (unsigned)std::min<long>(outer, 65535)), dim3(256), 0,
                         st, it, da, db, alpha, in, beta, out);
      return hipGetLastError();
    }
  }
  if (it.total < (1L << 32))
    hipLaunchKernelGGL((strided_axpby<TO, TI, unsigned>), dim3(blocks_for(it.total)), dim3(kThreads), 0, st, it,
                       alpha, in, beta, out);
  else
    hipLaunchKernelGGL((strided_axpby<TO, TI, unsigned long>), dim3(blocks_for(it.total)), dim3(kThreads), 0, st,
                       it, alpha, in, beta, out);
  return hipGetLastError();
}

hipError_t strided_copy(const Iter& it, double alpha, const double* in, double beta, double* out, hipStream_t st) {
  return launch_strided<double, double>(it, alpha, in, beta, out, st);
}

hipError_t strided_copy_f32(const Iter& it, double alpha, const double* in, float* out, hipStream_t st) {
  return launch_strided<float, double>(it, alpha, in, 0.0, out, st);
}

hipError_t fill(double* p, long n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, st, p, n, v);
  return hipGetLastError();
}

hipError_t symmetrize_pairs_scaled(double* x, int nh, int np, double scale, hipStream_t st) {
  if (nh <= 0 || np <= 0) return hipSuccess;
  const int nt = (np + kSymTile - 1) / kSymTile;
  const long pairs = (long)nh * (nh + 1) / 2;
  hipLaunchKernelGGL(symmetrize_kernel, dim3(nt * nt, (unsigned)std::min<long>(pairs, 65535)), dim3(256), 0, st, x,
                     nh, np, scale);
  return hipGetLastError();
}

hipError_t symmetrize_pairs(double* x, int nh, int np, hipStream_t st) {
  return symmetrize_pairs_scaled(x, nh, np, 1.0, st);
}

hipError_t lambda_update(double* l1, double* l2, const double* g1, const double* g2, const double* j1,
                         const double* j2, const double* eps, int nc, int na, int nv, double s, double* partial,
                         double* norm2, hipStream_t st) {
  hipLaunchKernelGGL(lambda_kernel, dim3(kRedBlocks), dim3(kThreads), 0, st, l1, l2, g1, g2, j1, j2, eps, nc, na, nv,
                     s, partial);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(kThreads), 0, st, partial, kRedBlocks, 1.0, norm2, 0);
  return hipGetLastError();
}

hipError_t flow_scale(const double* l1, const double* l2, const double* eps, int nc, int na, int nv, double s,
                      double* o1, double* o2, hipStream_t st) {
  const long n = (long)(nc + na) * (na + nv) * (1 + (long)(nc + na) * (na + nv));
  hipLaunchKernelGGL(flow_scale_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, st, l1, l2, eps, nc, na, nv, s, o1,
                     o2);
  return hipGetLastError();
}

hipError_t flow_fock_gradient(const double* t1, const double* t2, const double* r1, const double* r2,
                              const double* l1, const double* l2, const double* eps, int nc, int na, int nv,
                              double s, double* df, hipStream_t st) {
  const int n = nc + na + nv;
  hipLaunchKernelGGL(flow_fock_kernel, dim3(n), dim3(kThreads), 0, st, t1, t2, r1, r2, l1, l2, eps, nc, na, nv, s,
                     df);
  return hipGetLastError();
}

hipError_t fock_weights(double* w, int n, int nc, int na, const double* g1, hipStream_t st) {
  const long total = (long)n * n;
  hipLaunchKernelGGL(fock_weights_kernel, dim3(blocks_for(total)), dim3(kThreads), 0, st, w, n, nc, na, g1);
  return hipGetLastError();
}

hipError_t column_dot(const double* B, const double* d, int nx, long n2, double alpha, double* out, hipStream_t st) {
  hipLaunchKernelGGL(column_dot_kernel, dim3(blocks_for(n2)), dim3(kThreads), 0, st, B, d, nx, n2, alpha, out);
  return hipGetLastError();
}

hipError_t mask_active(double* r1, double* r2, int nc, int na, int nv, hipStream_t st) {
  const long n = (long)na * na * na * na + (long)na * na;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(mask_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, st, r1, r2, nc, na, nc + na, na + nv);
  return hipGetLastError();
}

hipError_t dot_accumulate(const double* a, const double* b, long n, double alpha, double* out, double* partial,
                          hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(dot_partial, dim3(kRedBlocks), dim3(kThreads), 0, st, a, b, n, partial);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(kThreads), 0, st, partial, kRedBlocks, alpha, out, 1);
  return hipGetLastError();
}

hipError_t ric_update_kernel(double* t1, double* t2, const double* r1, const double* r2, const double* eps, int nc,
                             int na, int nv, double s, double* partial, double* norm2, hipStream_t st) {
  hipLaunchKernelGGL(update_kernel, dim3(kRedBlocks), dim3(kThreads), 0, st, t1, t2, r1, r2, eps, nc, na, nv, s,
                     partial);
  hipLaunchKernelGGL(finish_sum, dim3(1), dim3(kThreads), 0, st, partial, kRedBlocks, 1.0, norm2, 0);
  return hipGetLastError();
}

hipError_t column_signs(double* u, int m, long ld, hipStream_t st) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(column_sign_kernel, dim3(m), dim3(kThreads), 0, st, u, m, ld);
  return hipGetLastError();
}

hipError_t fock_diagonal(const double* f, int n, double* eps, hipStream_t st) {
  hipLaunchKernelGGL(diag_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, st, f, n, eps);
  return hipGetLastError();
}

hipError_t check_finite(const double* x, long n, int* flag, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(nonfinite_kernel, dim3(blocks_for(n)), dim3(kThreads), 0, st, x, n, flag);
  return hipGetLastError();
}

hipError_t prepare_cumulants(const double* g1, const double* g2, const double* g3, int na, double* ga, double* ea,
                             double* l2, double* k2, double* l3, double* k3, hipStream_t st) {
  if (na <= 0) return hipSuccess;
  const long n4 = (long)na * na * na * na, n6 = n4 * na * na;
  hipLaunchKernelGGL(onebody_kernel, dim3(blocks_for(na * na)), dim3(kThreads), 0, st, g1, na, ga, ea);
  hipLaunchKernelGGL(lambda2_kernel, dim3(blocks_for(n4)), dim3(kThreads), 0, st, g1, g2, na, l2);
  hipLaunchKernelGGL(k2_kernel, dim3(blocks_for(n4)), dim3(kThreads), 0, st, l2, na, k2);
  hipLaunchKernelGGL(lambda3_kernel, dim3(blocks_for(n6)), dim3(kThreads), 0, st, g1, l2, g3, na, l3);
  hipLaunchKernelGGL(k3_kernel, dim3(blocks_for(n6)), dim3(kThreads), 0, st, l3, na, k3);
  return hipGetLastError();
}

hipError_t reference_energy(const double* f, int n, const double* I4, int nc, int na, const double* g1,
                            const double* g2, double* out, hipStream_t st) {
  hipLaunchKernelGGL(e0_kernel, dim3(1), dim3(kThreads), 0, st, f, n, I4, nc, na, g1, g2, out);
  return hipGetLastError();
}

hipError_t pack_tau(const double* tau, int nh, int np, double* tp, double* tm, long ldp, long ldm, hipStream_t st) {
  const long n = (long)nh * (nh + 1) / 2 * ldp + (long)nh * (nh - 1) / 2 * ldm;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((pack_tau_kernel<double>), dim3(blocks_for(n)), dim3(kThreads), 0, st, tau, nh, np, tp, tm, ldp,
                     ldm);
  return hipGetLastError();
}

hipError_t pack_tau_f32(const double* tau, int nh, int np, float* tp, float* tm, long ldp, long ldm, hipStream_t st) {
  const long n = (long)nh * (nh + 1) / 2 * ldp + (long)nh * (nh - 1) / 2 * ldm;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL((pack_tau_kernel<float>), dim3(blocks_for(n)), dim3(kThreads), 0, st, tau, nh, np, tp, tm, ldp,
                     ldm);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_pack_w(const T* w, int np, int rows, int c1, T* wp, T* wm, long ldp, long ldm,
                                hipStream_t st) {
  const long pairs = (long)rows * c1;
  if (pairs <= 0 || np <= 0) return hipSuccess;
  const int nt = (np + kPackTile - 1) / kPackTile;
  const unsigned gy = (unsigned)std::min<long>(pairs, 65535);
  hipLaunchKernelGGL((pack_w_kernel<T>), dim3(nt * (nt + 1) / 2, gy), dim3(256), 0, st, w, np, pairs, c1, wp, wm,
                     ldp, ldm);
  return hipGetLastError();
}

hipError_t pack_w(const double* w, int np, int rows, int c1, double* wp, double* wm, long ldp, long ldm,
                  hipStream_t st) {
  return launch_pack_w(w, np, rows, c1, wp, wm, ldp, ldm, st);
}

hipError_t pack_w_f32(const float* w, int np, int rows, int c1, float* wp, float* wm, long ldp, long ldm,
                      hipStream_t st) {
  return launch_pack_w(w, np, rows, c1, wp, wm, ldp, ldm, st);
}

hipError_t ladder_scatter_pm_add(const double* sp, const double* sm, int nh, int np, int c0, int c1, double* r2,
                                 hipStream_t st) {
  const long n = (long)nh * (nh + 1) / 2 * ((long)(c1 - c0) * c1);
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ladder_scatter_pm, dim3(blocks_for(n)), dim3(kThreads), 0, st, sp, sm, nh, np, c0, c1, r2);
  return hipGetLastError();
}

hipError_t ladder_scatter_add(const double* C, int nh, int np, int c0, int c1, int ncol, double* r2, hipStream_t st) {
  const long n = (long)nh * nh * (c1 - c0) * ncol;
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(ladder_scatter, dim3(blocks_for(n)), dim3(kThreads), 0, st, C, nh, np, c0, c1, ncol, r2);
  return hipGetLastError();
}

}  // namespace ric
