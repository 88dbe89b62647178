// Block CG kernels for gfx950 (generic path).
//
// One iteration of Algorithm 1 (Section 3, M = I) is three row-parallel
// passes over the n x k block vectors (row-major, k fastest) plus small
// reductions and solves:
//   spmm_product : Q = A P                      and partial alpha = <<P, Q>>_S
//   solve_lambda : lambda = sym(alpha)^{-1} rho  (Cholesky per group)
//   update_r     : R -= Q lambda                and partial <<R, R>>_S, ||R_j||^2
//   conv_beta    : stop rule, beta = rho^{-1} rho_new (LU with partial pivoting)
//   update_xp    : X += P lambda, P = R + P beta and partial rho = <<P, R>>_S
// (X is updated in the pass that reads P anyway, one kernel after R),
// so every block product is accumulated by the kernel that produces its
// operands (the paper notes the recomputed rho can share a reduction with the
// product before it, Section 3). The partial products of each workgroup are
// summed in a fixed order by `reduce`, so results are bitwise reproducible.
//
// Block products <<X, Y>>_S (Section 2): the q diagonal p x p blocks
// X_g^T Y_g of X^T Y (hybrid / block / parallel), or their sum (global), in
// the packed layout [qo][p][p].
#include <algorithm>
#include <cfloat>
#include <type_traits>
#include <cmath>

#include "../../include/bcg.h"
#include "bcg_internal.h"
#include "bcg_scale.h"

namespace bcg {

namespace {

__device__ __forceinline__ bool stopped(const DevState* st) {
  return st != nullptr && *reinterpret_cast<const volatile int*>(&st->done) != 0;
}

__device__ __forceinline__ void set_status(DevState* st, int status) {
  *reinterpret_cast<volatile int*>(&st->status) = status;
  *reinterpret_cast<volatile int*>(&st->done) = 1;
}

// The iteration that just updated R is the last one: X still receives its
// P lambda in the X/P pass.
__device__ __forceinline__ void set_last(DevState* st, int status) {
  *reinterpret_cast<volatile int*>(&st->status) = status;
  *reinterpret_cast<volatile int*>(&st->last) = 1;
}

// ------------------------------------------------------------------------
// Block-product accumulation over LDS tiles.
//
// Entry block eb = (g, A, Bb) owns the RB x RB entries
// (a, b) = (A*RB + i, Bb*RB + j) of packed block g. When there are fewer
// entry blocks than threads, the rows of a tile are split into S slices.
// ------------------------------------------------------------------------
template <int RB, int NAB>
struct Acc {
  double v[NAB][RB][RB];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int j = 0; j < NAB; ++j)
#pragma unroll
      for (int a = 0; a < RB; ++a)
#pragma unroll
        for (int b = 0; b < RB; ++b) v[j][a][b] = 0.0;
  }
};

__device__ __forceinline__ void decode_eb(const Plan& pl, int eb, int& g, int& A, int& Bb) {
  const int pp = pl.pb * pl.pb;
  g = eb / pp;
  const int r = eb - g * pp;
  A = r / pl.pb;
  Bb = r - A * pl.pb;
}

template <typename T, int RB>
__device__ __forceinline__ void acc_rows(double (&acc)[RB][RB], const T* Xs, const T* Ys, const Plan& pl,
                                         int g, int A, int Bb, int r0, int rows, int rstep) {
  const int k = pl.k, p = pl.p;
  const int g0 = pl.global ? 0 : g;
  const int g1 = pl.global ? pl.q : g + 1;
  for (int r = r0; r < rows; r += rstep) {
    const T* xr = Xs + r * k + A * RB;
    const T* yr = Ys + r * k + Bb * RB;
    for (int gg = g0; gg < g1; ++gg) {
      double x[RB], y[RB];
#pragma unroll
      for (int i = 0; i < RB; ++i) {
        x[i] = static_cast<double>(xr[gg * p + i]);
        y[i] = static_cast<double>(yr[gg * p + i]);
      }
#pragma unroll
      for (int i = 0; i < RB; ++i)
#pragma unroll
        for (int j = 0; j < RB; ++j) acc[i][j] = fma(x[i], y[j], acc[i][j]);
    }
  }
}

// Accumulates entry blocks [eb_off, eb_lim) of <<Xs, Ys>> over `rows` rows.
template <typename T, int RB, int NAB>
__device__ __forceinline__ void product_tile(Acc<RB, NAB>& acc, const T* Xs, const T* Ys, int rows,
                                             const Plan& pl, int tid, int eb_off, int eb_lim) {
  if (pl.EB <= kBlock) {
    if (tid < pl.S * pl.EB) {
      const int eb = tid % pl.EB, s = tid / pl.EB;
      int g, A, Bb;
      decode_eb(pl, eb, g, A, Bb);
      acc_rows<T, RB>(acc.v[0], Xs, Ys, pl, g, A, Bb, s, rows, pl.S);
    }
  } else {
#pragma unroll
    for (int j = 0; j < NAB; ++j) {
      const int eb = eb_off + tid + j * kBlock;
      if (eb < eb_lim) {
        int g, A, Bb;
        decode_eb(pl, eb, g, A, Bb);
        acc_rows<T, RB>(acc.v[j], Xs, Ys, pl, g, A, Bb, 0, rows, 1);
      }
    }
  }
}

// Writes the workgroup's partial product (slices summed in a fixed order).
template <int RB, int NAB>
__device__ void product_finish(const Acc<RB, NAB>& acc, double* prow, const Plan& pl, double* scratch,
                               int tid, int eb_off, int eb_lim) {
  const int p = pl.p;
  if (pl.EB <= kBlock) {
    const bool active = tid < pl.S * pl.EB;
#pragma unroll
    for (int i = 0; i < RB; ++i)
#pragma unroll
      for (int j = 0; j < RB; ++j) scratch[(tid * RB + i) * RB + j] = active ? acc.v[0][i][j] : 0.0;
    __syncthreads();
    if (tid < pl.EB) {
      int g, A, Bb;
      decode_eb(pl, tid, g, A, Bb);
      for (int i = 0; i < RB; ++i)
        for (int j = 0; j < RB; ++j) {
          double s = 0.0;
          for (int sl = 0; sl < pl.S; ++sl) s += scratch[((sl * pl.EB + tid) * RB + i) * RB + j];
          prow[(int64_t)g * p * p + (A * RB + i) * p + Bb * RB + j] = s;
        }
    }
    __syncthreads();
  } else {
#pragma unroll
    for (int jb = 0; jb < NAB; ++jb) {
      const int eb = eb_off + tid + jb * kBlock;
      if (eb < eb_lim) {
        int g, A, Bb;
        decode_eb(pl, eb, g, A, Bb);
#pragma unroll
        for (int i = 0; i < RB; ++i)
#pragma unroll
          for (int j = 0; j < RB; ++j) prow[(int64_t)g * p * p + (A * RB + i) * p + Bb * RB + j] = acc.v[jb][i][j];
      }
    }
  }
}

// Column sums of squares of an LDS tile (k <= kBlock).
template <typename T>
__device__ __forceinline__ void norms_tile(double& acc, const T* Rs, int rows, int k, int tid) {
  const int sn = kBlock / k;
  if (tid < sn * k) {
    const int c = tid % k, s = tid / k;
    for (int r = s; r < rows; r += sn) {
      const double v = static_cast<double>(Rs[r * k + c]);
      acc = fma(v, v, acc);
    }
  }
}

__device__ void norms_finish(double acc, double* out, int k, double* scratch, int tid) {
  scratch[tid] = acc;
  __syncthreads();
  if (tid < k) {
    const int sn = kBlock / k;
    double s = 0.0;
    for (int sl = 0; sl < sn; ++sl) s += scratch[sl * k + tid];
    out[tid] = s;
  }
  __syncthreads();
}

struct TileRange {
  int64_t row0, base;
  int rows, ne;
};

__device__ __forceinline__ TileRange tile_range(const Plan& pl, int64_t t) {
  TileRange tr;
  tr.row0 = t * pl.TR;
  const int64_t left = pl.n - tr.row0;
  tr.rows = static_cast<int>(left < pl.TR ? left : pl.TR);
  tr.ne = tr.rows * pl.k;
  tr.base = tr.row0 * pl.k;
  return tr;
}

// ------------------------------------------------------------------------
// Row kernels
// ------------------------------------------------------------------------

// R = B - A X (FP64); P = R and <<R, R>> partial when with_p; column norms.
template <int RB, int NAB>
__global__ __launch_bounds__(kBlock) void k_residual(Plan pl, const int32_t* __restrict__ rowptr,
                                                     const int32_t* __restrict__ colind,
                                                     const double* __restrict__ vals,
                                                     const double* __restrict__ B, const double* __restrict__ X,
                                                     double* __restrict__ R, double* __restrict__ P,
                                                     double* __restrict__ part, int with_p) {
  __shared__ double Rs[kTileElems];
  __shared__ double scratch[kBlock * RB * RB];
  const int tid = threadIdx.x, k = pl.k;
  Acc<RB, NAB> acc;
  acc.zero();
  double nacc = 0.0;
  const bool prod = with_p && pl.fused;
  for (int64_t t = blockIdx.x; t < pl.ntiles; t += gridDim.x) {
    const TileRange tr = tile_range(pl, t);
    for (int e = tid; e < tr.ne; e += kBlock) {
      const int r = e / k, c = e - r * k;
      const int64_t i = tr.row0 + r;
      // entries in chunks of 8: all index and value loads, then all gathers,
      // then the products in entry order (an entry past the row end adds
      // 0 * x for a clamped, valid column, which leaves s unchanged)
      double s = 0.0;
      const int j0 = rowptr[i], j1 = rowptr[i + 1];
      for (int jb = j0; jb < j1; jb += 8) {
        int cols[8];
        double vs[8], xs[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int jj = min(jb + u, j1 - 1);
          cols[u] = colind[jj];
          vs[u] = jb + u < j1 ? vals[jj] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) xs[u] = X[(int64_t)cols[u] * k + c];
#pragma unroll
        for (int u = 0; u < 8; ++u) s = fma(vs[u], xs[u], s);
      }
      const double v = B[tr.base + e] - s;
      R[tr.base + e] = v;
      if (with_p) P[tr.base + e] = v;
      Rs[e] = v;
    }
    __syncthreads();
    if (prod) product_tile<double, RB, NAB>(acc, Rs, Rs, tr.rows, pl, tid, 0, pl.EB);
    norms_tile<double>(nacc, Rs, tr.rows, k, tid);
    __syncthreads();
  }
  double* prow = part + (int64_t)blockIdx.x * pl.W;
  if (prod) product_finish<RB, NAB>(acc, prow, pl, scratch, tid, 0, pl.EB);
  norms_finish(nacc, prow + pl.E, k, scratch, tid);
}

// FP32 inner start of a refinement step.
template <int RB, int NAB>
// R32 = R64 / s with s = max_j sqrt(norms[j]) (stored to *scale), D32 = 0,
// and P32 = R32 (pfac = 0: a fresh start) or P32 *= pfac rounded to FP32
// (pfac != 0: the search direction in the units of the new scale, residual
// replacement); the partial <<R32, R32>> with the column norms.
__global__ __launch_bounds__(kBlock) void k_cast_init(Plan pl, const double* __restrict__ R64,
                                                      const double* __restrict__ norms, float* __restrict__ R32,
                                                      float* __restrict__ P32, float* __restrict__ D32,
                                                      double* __restrict__ scale, double* __restrict__ part,
                                                      double pfac) {
  __shared__ float Rs[kTileElems];
  __shared__ double scratch[kBlock * RB * RB];
  __shared__ double s_sh;
  const int tid = threadIdx.x, k = pl.k;
  if (tid == 0) {
    double m = 0.0;
    for (int j = 0; j < k; ++j) m = fmax(m, sqrt(norms[j]));
    s_sh = m;
    if (blockIdx.x == 0) *scale = m;
  }
  __syncthreads();
  const double s = s_sh;
  Acc<RB, NAB> acc;
  acc.zero();
  double nacc = 0.0;
  for (int64_t t = blockIdx.x; t < pl.ntiles; t += gridDim.x) {
    const TileRange tr = tile_range(pl, t);
    for (int e = tid; e < tr.ne; e += kBlock) {
      const float v = static_cast<float>(R64[tr.base + e] / s);
      R32[tr.base + e] = v;
      P32[tr.base + e] = pfac == 0.0 ? v : P32[tr.base + e] * static_cast<float>(pfac);
      D32[tr.base + e] = 0.0f;
      Rs[e] = v;
    }
    __syncthreads();
    if (pl.fused) product_tile<float, RB, NAB>(acc, Rs, Rs, tr.rows, pl, tid, 0, pl.EB);
    norms_tile<float>(nacc, Rs, tr.rows, k, tid);
    __syncthreads();
  }
  double* prow = part + (int64_t)blockIdx.x * pl.W;
  if (pl.fused) product_finish<RB, NAB>(acc, prow, pl, scratch, tid, 0, pl.EB);
  norms_finish(nacc, prow + pl.E, k, scratch, tid);
}

// Q = A P and the partial alpha = <<P, Q>>.
template <typename T, int RB, int NAB>
__global__ __launch_bounds__(kBlock) void k_spmm_product(Plan pl, const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colind,
                                                         const T* __restrict__ vals, const T* __restrict__ P,
                                                         T* __restrict__ Q, double* __restrict__ part,
                                                         const DevState* st) {
  if (halted(st)) return;
  __shared__ T Ps[kTileElems];
  __shared__ T Qs[kTileElems];
  __shared__ double scratch[kBlock * RB * RB];
  const int tid = threadIdx.x, k = pl.k;
  Acc<RB, NAB> acc;
  acc.zero();
  for (int64_t t = blockIdx.x; t < pl.ntiles; t += gridDim.x) {
    const TileRange tr = tile_range(pl, t);
    for (int e = tid; e < tr.ne; e += kBlock) {
      const int r = e / k, c = e - r * k;
      const int64_t i = pl.sched ? static_cast<int64_t>(pl.sched[tr.row0 + r]) : tr.row0 + r;
      T s = T(0);
      const int j1 = rowptr[i + 1];
      for (int j = rowptr[i]; j < j1; ++j) s = fma(vals[j], P[(int64_t)colind[j] * k + c], s);
      Q[i * k + c] = s;
      Qs[e] = s;
      Ps[e] = P[i * k + c];
    }
    __syncthreads();
    if (pl.fused) product_tile<T, RB, NAB>(acc, Ps, Qs, tr.rows, pl, tid, 0, pl.EB);
    __syncthreads();
  }
  if (pl.fused) product_finish<RB, NAB>(acc, part + (int64_t)blockIdx.x * pl.W, pl, scratch, tid, 0, pl.EB);
}

// R -= Q lambda (line 9); partial <<R, R>> and column norms of R.
template <typename T, int RB, int NAB>
__global__ __launch_bounds__(kBlock) void k_update_r(Plan pl, T* __restrict__ R, const T* __restrict__ Q,
                                                     const T* __restrict__ lam, double* __restrict__ part,
                                                     const DevState* st) {
  if (stopped(st)) return;
  __shared__ T Qs[kTileElems];
  __shared__ T Rs[kTileElems];
  __shared__ T lamS[kLamLds];
  __shared__ double scratch[kBlock * RB * RB];
  const int tid = threadIdx.x, k = pl.k, p = pl.p;
  const bool lds_lam = pl.E <= kLamLds;
  if (lds_lam)
    for (int e = tid; e < pl.E; e += kBlock) lamS[e] = lam[e];
  const T* L = lds_lam ? lamS : lam;
  Acc<RB, NAB> acc;
  acc.zero();
  double nacc = 0.0;
  for (int64_t t = blockIdx.x; t < pl.ntiles; t += gridDim.x) {
    const TileRange tr = tile_range(pl, t);
    for (int e = tid; e < tr.ne; e += kBlock) Qs[e] = Q[tr.base + e];
    __syncthreads();
    for (int e = tid; e < tr.ne; e += kBlock) {
      const int r = e / k, c = e - r * k;
      const int g = c / p, b = c - g * p;
      const T* lg = L + (pl.global ? 0 : g * p * p) + b;
      const T* qr = Qs + r * k + g * p;
      T dr = T(0);
      for (int a = 0; a < p; ++a) dr = fma(qr[a], lg[a * p], dr);
      const T rn = R[tr.base + e] - dr;
      R[tr.base + e] = rn;
      Rs[e] = rn;
    }
    __syncthreads();
    if (pl.fused) product_tile<T, RB, NAB>(acc, Rs, Rs, tr.rows, pl, tid, 0, pl.EB);
    norms_tile<T>(nacc, Rs, tr.rows, k, tid);
    __syncthreads();
  }
  double* prow = part + (int64_t)blockIdx.x * pl.W;
  if (pl.fused) product_finish<RB, NAB>(acc, prow, pl, scratch, tid, 0, pl.EB);
  norms_finish(nacc, prow + pl.E, k, scratch, tid);
}

// X += P lambda (line 8); unless last: P = R + P beta (line 13) and the
// partial rho = <<P_new, R>> for the next iteration's line 6.
template <typename T, int RB, int NAB>
__global__ __launch_bounds__(kBlock) void k_update_xp(Plan pl, T* __restrict__ X, T* __restrict__ P,
                                                      const T* __restrict__ R, const T* __restrict__ lam,
                                                      const T* __restrict__ beta, double* __restrict__ part,
                                                      const DevState* st) {
  if (stopped(st)) return;
  const bool last = *reinterpret_cast<const volatile int*>(&st->last) != 0;
  __shared__ T Ps[kTileElems];
  __shared__ T Rs[kTileElems];
  __shared__ T Pn[kTileElems];
  __shared__ T cS[2 * kLamLds];
  __shared__ double scratch[kBlock * RB * RB];
  const int tid = threadIdx.x, k = pl.k, p = pl.p;
  const bool lds_c = pl.E <= kLamLds;
  if (lds_c)
    for (int e = tid; e < pl.E; e += kBlock) {
      cS[e] = lam[e];
      if (!last) cS[kLamLds + e] = beta[e];
    }
  const T* L = lds_c ? cS : lam;
  const T* Bt = lds_c ? cS + kLamLds : beta;
  Acc<RB, NAB> acc;
  acc.zero();
  for (int64_t t = blockIdx.x; t < pl.ntiles; t += gridDim.x) {
    const TileRange tr = tile_range(pl, t);
    for (int e = tid; e < tr.ne; e += kBlock) {
      Ps[e] = P[tr.base + e];
      if (!last) Rs[e] = R[tr.base + e];
    }
    __syncthreads();
    for (int e = tid; e < tr.ne; e += kBlock) {
      const int r = e / k, c = e - r * k;
      const int g = c / p, b = c - g * p;
      const int off = (pl.global ? 0 : g * p * p) + b;
      const T* pr = Ps + r * k + g * p;
      T dx = T(0), dp = T(0);
      for (int a = 0; a < p; ++a) dx = fma(pr[a], L[off + a * p], dx);
      X[tr.base + e] += dx;
      if (!last) {
        for (int a = 0; a < p; ++a) dp = fma(pr[a], Bt[off + a * p], dp);
        const T pn = Rs[e] + dp;
        P[tr.base + e] = pn;
        Pn[e] = pn;
      }
    }
    __syncthreads();
    if (pl.fused && !last) product_tile<T, RB, NAB>(acc, Pn, Rs, tr.rows, pl, tid, 0, pl.EB);
    __syncthreads();
  }
  if (pl.fused) product_finish<RB, NAB>(acc, part + (int64_t)blockIdx.x * pl.W, pl, scratch, tid, 0, pl.EB);
}

// Stand-alone product of global X, Y for entry blocks [eb_off, eb_off + NAB*kBlock).
template <typename T, int RB, int NAB>
__global__ __launch_bounds__(kBlock) void k_product(Plan pl, const T* __restrict__ X, const T* __restrict__ Y,
                                                    double* __restrict__ part, const DevState* st, int eb_off) {
  if (stopped(st)) return;
  __shared__ T Xs[kTileElems];
  __shared__ T Ys[kTileElems];
  __shared__ double scratch[kBlock * RB * RB];
  const int tid = threadIdx.x;
  const int eb_lim = min(pl.EB, eb_off + NAB * kBlock);
  Acc<RB, NAB> acc;
  acc.zero();
  for (int64_t t = blockIdx.x; t < pl.ntiles; t += gridDim.x) {
    const TileRange tr = tile_range(pl, t);
    for (int e = tid; e < tr.ne; e += kBlock) {
      Xs[e] = X[tr.base + e];
      Ys[e] = Y[tr.base + e];
    }
    __syncthreads();
    product_tile<T, RB, NAB>(acc, Xs, Ys, tr.rows, pl, tid, eb_off, eb_lim);
    __syncthreads();
  }
  product_finish<RB, NAB>(acc, part + (int64_t)blockIdx.x * pl.W, pl, scratch, tid, eb_off, eb_lim);
}

// ------------------------------------------------------------------------
// Reductions and small solves
// ------------------------------------------------------------------------

// out[e] = sum over partial rows w in [r0, r1) of part[w][e] for the EPB
// entries e = EPB b .. EPB b + EPB - 1 below width, in a fixed order: the
// block's SLOTS thread slots each take every SLOTS-th partial row (term t of
// slot s is row r0 + s + SLOTS t, summed into chain t mod 4; the loads of 32
// terms are issued together), and a fixed tree combines the slot sums.
// Every thread of the block (SLOTS * EPB threads) calls it; wave 0 makes the
// stores.
constexpr int kRedThreads = 1024;
constexpr int kRedBatch = 32;

template <int EPB, int SLOTS>
__device__ __forceinline__ void reduce_entries(const double* __restrict__ part, double* __restrict__ out, int width,
                                               int W, int r0, int r1, int b, double (*sh)[EPB]) {
  static_assert(EPB <= 64, "the stores come from wave 0");
  const int tid = threadIdx.x, le = tid % EPB, s = tid / EPB;
  const int e = b * EPB + le;
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  if (e < width) {
    // byte offset of (row r0 + s, entry e) from the base of the batch (below
    // 2^32: s < SLOTS rows of at most 65792 entries); the steps of SLOTS
    // rows go into the uniform base
    const uint32_t off = (static_cast<uint32_t>(s) * static_cast<uint32_t>(W) + static_cast<uint32_t>(e)) * 8u;
    const size_t step = static_cast<size_t>(W) * SLOTS * sizeof(double);
    for (int t0 = 0; r0 + s + SLOTS * t0 < r1; t0 += kRedBatch) {
      const char* base = reinterpret_cast<const char*>(part + (int64_t)r0 * W) + step * t0;
      double v[kRedBatch];
#pragma unroll
      for (int t = 0; t < kRedBatch; ++t)
        v[t] = r0 + s + SLOTS * (t0 + t) < r1 ? *reinterpret_cast<const double*>(base + step * t + off) : 0.0;
#pragma unroll
      for (int t = 0; t < kRedBatch; ++t) c[t & 3] += v[t];
    }
  }
  sh[s][le] = (c[0] + c[1]) + (c[2] + c[3]);
  __syncthreads();
  for (int h = SLOTS / 2; h > 0; h >>= 1) {
    if (s < h) sh[s][le] = sh[s][le] + sh[s + h][le];
    __syncthreads();
  }
  if (s == 0 && e < width) out[e] = sh[0][le];  // wave 0 (tid < EPB) stores
}

__global__ __launch_bounds__(kRedThreads) void k_reduce(const double* __restrict__ part, double* __restrict__ out,
                                                        int width, int W, int nwg, const DevState* st) {
  if (stopped(st)) return;
  __shared__ double sh[64][16];
  reduce_entries<16, 64>(part, out, width, W, 0, nwg, blockIdx.x, sh);
}

// First stage for many partial rows: block (b, q) sums split q of the rows
// (rows r0..r1-1) for 64 consecutive entries into row q of `out` (kRedSplits
// rows of stride W); a second pass then sums the kRedSplits rows. Each wave
// reads 512 contiguous bytes of a row per load, and a thread keeps 8 loads in
// flight; thread slot s sums rows r0 + s, r0 + s + 4, ... in that order, and
// the four slots are added in a fixed order, so the sums are reproducible.
constexpr int kRowsEPB = 64, kRowsSlots = 4, kRowsBatch = 8;
constexpr int kRowsThreads = kRowsEPB * kRowsSlots;
__global__ __launch_bounds__(kRowsThreads) void k_reduce_rows(const double* __restrict__ part,
                                                              double* __restrict__ out, int width, int W, int rows,
                                                              const DevState* st) {
  if (stopped(st)) return;
  __shared__ double sh[kRowsSlots][kRowsEPB];
  const int q = blockIdx.y;
  const int r0 = static_cast<int>(static_cast<int64_t>(rows) * q / kRedSplits);
  const int r1 = static_cast<int>(static_cast<int64_t>(rows) * (q + 1) / kRedSplits);
  const int le = threadIdx.x % kRowsEPB, s = threadIdx.x / kRowsEPB;
  const int e = blockIdx.x * kRowsEPB + le;
  double c[4] = {0.0, 0.0, 0.0, 0.0};
  if (e < width) {
    const int64_t step = static_cast<int64_t>(W) * kRowsSlots;
    const double* p = part + static_cast<int64_t>(r0 + s) * W + e;
    int r = r0 + s;
    for (; r + (kRowsBatch - 1) * kRowsSlots < r1; r += kRowsBatch * kRowsSlots, p += kRowsBatch * step) {
      double v[kRowsBatch];
#pragma unroll
      for (int t = 0; t < kRowsBatch; ++t) v[t] = p[t * step];
#pragma unroll
      for (int t = 0; t < kRowsBatch; ++t) c[t & 3] += v[t];
    }
    for (; r < r1; r += kRowsSlots, p += step) c[0] += *p;
  }
  sh[s][le] = (c[0] + c[1]) + (c[2] + c[3]);
  __syncthreads();
  if (s == 0 && e < width) out[(int64_t)q * W + e] = (sh[0][le] + sh[1][le]) + (sh[2][le] + sh[3][le]);
}

// True in the one workgroup of the launch that finishes its share last; its
// loads after the call see the stores of every workgroup. Wave 0 must have
// made all of the workgroup's global stores (as reduce_entries does): its
// release fence orders them before the ticket, so no other wave pays for a
// fence. The last workgroup resets the ticket for the next launch. Every
// thread calls it.
__device__ __forceinline__ bool last_workgroup(DevState* st) {
  __shared__ int is_last;
  if (threadIdx.x < 64) {
    __threadfence();  // this wave's stores before the ticket
    if (threadIdx.x == 0) {
      const unsigned int t = atomicAdd(&st->ticket, 1u);
      is_last = t == gridDim.x * gridDim.y - 1;
      if (is_last) {
        atomicExch(&st->ticket, 0u);
        __threadfence();  // the other workgroups' stores before the loads that follow
      }
    }
  }
  __syncthreads();
  return is_last;
}

constexpr int kSmallLdsP = 48;  // p x p solves of up to this size run in LDS

// lambda_g = sym(alpha_g)^{-1} rho_g by Cholesky (Algorithm 1 line 7).
__global__ __launch_bounds__(kBlock) void k_solve_lambda(Plan pl, const double* __restrict__ alpha,
                                                         const double* __restrict__ rho, double* __restrict__ lam,
                                                         float* __restrict__ lam32, double* __restrict__ ws,
                                                         DevState* st) {
  if (stopped(st)) return;
  const int tid = threadIdx.x, p = pl.p;
  __shared__ int flag;
  if (p == 1) {
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int e = tid; e < pl.E; e += kBlock) {
      const double a = alpha[e], r = rho[e];
      double l = 0.0;
      if (pl.dec && a == 0.0 && r == 0.0) {
        l = 0.0;
      } else if (!(a > 0.0) || !isfinite(a)) {
        flag = 1;
      } else {
        l = r / a;
      }
      lam[e] = l;
      lam32[e] = static_cast<float>(l);
    }
    __syncthreads();
    if (tid == 0 && flag) set_status(st, BCG_EBREAKDOWN);
    return;
  }
  __shared__ double lds[2 * kSmallLdsP * kSmallLdsP];
  const int g = blockIdx.x, pp = p * p;
  double* M = (p <= kSmallLdsP) ? lds : ws + (int64_t)g * 2 * pp;
  double* Y = M + pp;
  const double* al = alpha + (int64_t)g * pp;
  const double* rh = rho + (int64_t)g * pp;
  if (tid == 0) flag = 0;
  __syncthreads();
  for (int e = tid; e < pp; e += kBlock) {
    const int i = e / p, j = e - i * p;
    const double m = 0.5 * (al[i * p + j] + al[j * p + i]);
    M[e] = m;
    Y[e] = rh[e];
    if (!isfinite(m) || !isfinite(rh[e])) flag = 1;
  }
  __syncthreads();
  // Cholesky, column by column; L overwrites the lower triangle of M.
  for (int j = 0; j < p && !flag; ++j) {
    if (tid == 0) {
      const double ajj = M[j * p + j];
      double s = 0.0;
      for (int m = 0; m < j; ++m) s = fma(M[j * p + m], M[j * p + m], s);
      const double d = ajj - s;
      if (!isfinite(d) || !(d > p * DBL_EPSILON * ajj) || !(ajj > 0.0))
        flag = 1;
      else
        M[j * p + j] = sqrt(d);
    }
    __syncthreads();
    if (flag) break;
    const double ljj = M[j * p + j];
    for (int i = j + 1 + tid; i < p; i += kBlock) {
      double s = 0.0;
      for (int m = 0; m < j; ++m) s = fma(M[i * p + m], M[j * p + m], s);
      M[i * p + j] = (M[i * p + j] - s) / ljj;
    }
    __syncthreads();
  }
  if (flag) {
    if (tid == 0) set_status(st, BCG_EBREAKDOWN);
    return;
  }
  for (int c = tid; c < p; c += kBlock) {
    for (int i = 0; i < p; ++i) {  // L y = rho
      double s = Y[i * p + c];
      for (int m = 0; m < i; ++m) s -= M[i * p + m] * Y[m * p + c];
      Y[i * p + c] = s / M[i * p + i];
    }
    for (int i = p - 1; i >= 0; --i) {  // L^T x = y
      double s = Y[i * p + c];
      for (int m = i + 1; m < p; ++m) s -= M[m * p + i] * Y[m * p + c];
      Y[i * p + c] = s / M[i * p + i];
    }
  }
  __syncthreads();
  double* lo = lam + (int64_t)g * pp;
  float* lo32 = lam32 + (int64_t)g * pp;
  for (int e = tid; e < pp; e += kBlock) {
    lo[e] = Y[e];
    lo32[e] = static_cast<float>(Y[e]);
  }
}

// Stop rule (Section 4 reading: every column's recursive residual norm below
// tol times its initial norm), then beta_g = rho_g^{-1} rho_new_g by LU with
// partial pivoting (Algorithm 1 lines 9-12).
__global__ __launch_bounds__(kBlock) void k_conv_beta(Plan pl, const double* __restrict__ red_new,
                                                      const double* __restrict__ r0,
                                                      const double* __restrict__ rho_old, double* __restrict__ beta,
                                                      float* __restrict__ beta32, double* __restrict__ ws,
                                                      double* __restrict__ ratios, DevState* st, double tol, int it,
                                                      int maxit) {
  if (stopped(st)) return;
  const int tid = threadIdx.x, k = pl.k, p = pl.p;
  __shared__ double smax[kBlock];
  __shared__ int sbad[kBlock];
  __shared__ int flag;
  double m = 0.0;
  int bad = 0;
  for (int j = tid; j < k; j += kBlock) {
    const double c = red_new[pl.E + j];
    const double rr = r0[j];
    const double ratio = (rr == 0.0) ? 0.0 : sqrt(c) / rr;
    if (!isfinite(ratio))
      bad = 1;
    else
      m = fmax(m, ratio);
    if (blockIdx.x == 0) ratios[j] = ratio;
  }
  smax[tid] = m;
  sbad[tid] = bad;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      smax[tid] = fmax(smax[tid], smax[tid + s]);
      sbad[tid] |= sbad[tid + s];
    }
    __syncthreads();
  }
  const bool lead = blockIdx.x == 0 && tid == 0;
  if (lead) {
    st->iter = it;
    st->max_ratio = sbad[0] ? NAN : smax[0];
  }
  if (sbad[0]) {
    if (lead) set_last(st, BCG_EBREAKDOWN);
    return;
  }
  if (smax[0] <= tol) {
    if (lead) set_last(st, BCG_OK);
    return;
  }
  if (it >= maxit) {
    if (lead) set_last(st, BCG_NOT_CONVERGED);
    return;
  }
  if (tid == 0) flag = 0;
  __syncthreads();
  if (p == 1) {
    for (int e = tid; e < pl.E; e += kBlock) {
      const double r = rho_old[e];
      double b = 0.0;
      if (pl.dec && r == 0.0) {
        b = 0.0;
      } else if (r == 0.0 || !isfinite(r)) {
        flag = 1;
      } else {
        b = red_new[e] / r;
      }
      beta[e] = b;
      beta32[e] = static_cast<float>(b);
    }
    __syncthreads();
    if (tid == 0 && flag) set_last(st, BCG_EBREAKDOWN);
    return;
  }
  __shared__ double lds[2 * kSmallLdsP * kSmallLdsP];
  __shared__ int piv;
  const int g = blockIdx.x, pp = p * p;
  double* M = (p <= kSmallLdsP) ? lds : ws + (int64_t)g * 2 * pp;
  double* Y = M + pp;
  for (int e = tid; e < pp; e += kBlock) {
    M[e] = rho_old[(int64_t)g * pp + e];
    Y[e] = red_new[(int64_t)g * pp + e];
    if (!isfinite(M[e])) flag = 1;
  }
  __syncthreads();
  for (int j = 0; j < p && !flag; ++j) {
    if (tid == 0) {
      int best_i = j;
      double best = fabs(M[j * p + j]);
      for (int i = j + 1; i < p; ++i) {
        const double v = fabs(M[i * p + j]);
        if (v > best) {
          best = v;
          best_i = i;
        }
      }
      if (best == 0.0) flag = 1;
      piv = best_i;
    }
    __syncthreads();
    if (flag) break;
    const int pr = piv;
    if (pr != j) {
      for (int c = tid; c < p; c += kBlock) {
        double t = M[j * p + c];
        M[j * p + c] = M[pr * p + c];
        M[pr * p + c] = t;
        t = Y[j * p + c];
        Y[j * p + c] = Y[pr * p + c];
        Y[pr * p + c] = t;
      }
      __syncthreads();
    }
    const double djj = M[j * p + j];
    const int rows = p - 1 - j;
    // eliminate below the pivot: columns j+1.. of M and all columns of Y
    for (int e = tid; e < rows * (2 * p); e += kBlock) {
      const int i = j + 1 + e / (2 * p);
      const int c = e % (2 * p);
      const double l = M[i * p + j] / djj;
      if (c < p) {
        if (c > j) M[i * p + c] -= l * M[j * p + c];
      } else {
        Y[i * p + (c - p)] -= l * Y[j * p + (c - p)];
      }
    }
    __syncthreads();
  }
  if (flag) {
    if (tid == 0) set_last(st, BCG_EBREAKDOWN);
    return;
  }
  for (int c = tid; c < p; c += kBlock) {
    for (int i = p - 1; i >= 0; --i) {
      double s = Y[i * p + c];
      for (int m2 = i + 1; m2 < p; ++m2) s -= M[i * p + m2] * Y[m2 * p + c];
      Y[i * p + c] = s / M[i * p + i];
    }
  }
  __syncthreads();
  for (int e = tid; e < pp; e += kBlock) {
    beta[(int64_t)g * pp + e] = Y[e];
    beta32[(int64_t)g * pp + e] = static_cast<float>(Y[e]);
  }
}

// ---- one wave per p x p group (p in {2, 4, 8, 16, 32}), rows in registers ----
// Lane i holds row i; the pivot row of each elimination step is broadcast
// with readlane, so the factorisations need no LDS round trips or barriers.

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ double readlane_d(double x, int l) {
  const long long v = __double_as_longlong(x);
  const int lo = __builtin_amdgcn_readlane(static_cast<int>(v & 0xffffffffLL), l);
  const int hi = __builtin_amdgcn_readlane(static_cast<int>(v >> 32), l);
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Value of lane (l - K) mod 16 within each row of 16 lanes (DPP row_ror:K).
template <int K>
__device__ __forceinline__ int ror16(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x120 + K, 0xF, 0xF, false);
}
template <int K>
__device__ __forceinline__ double ror16(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = ror16<K>(static_cast<int>(v & 0xffffffffLL));
  const int hi = ror16<K>(static_cast<int>(v >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// Maximum (NaN ignored, as by fmax) and minimum over each row of 16 lanes,
// left in every lane of the row.
__device__ __forceinline__ double row16_max(double v) {
  v = fmax(v, ror16<8>(v));
  v = fmax(v, ror16<4>(v));
  v = fmax(v, ror16<2>(v));
  return fmax(v, ror16<1>(v));
}
__device__ __forceinline__ int row16_min(int v) {
  v = min(v, ror16<8>(v));
  v = min(v, ror16<4>(v));
  v = min(v, ror16<2>(v));
  return min(v, ror16<1>(v));
}

// g itself, through a register the compiler cannot see into: keeps the
// addresses of one group's solve from being carried across the group loop
// (as one live pointer per access).
__device__ __forceinline__ int opaque(int g) {
  asm volatile("" : "+v"(g));
  return g;
}

// 0, as an offset the compiler cannot compute before v is.
__device__ __forceinline__ int after(double v) {
  int z = 0;
  asm volatile("" : "+v"(z) : "v"(v));
  return z;
}

// 1 / sqrt(d) for finite d > 0: the hardware estimate and two Newton steps
// (each squares the relative error), within an ulp or two.
__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int n = 0; n < 2; ++n) {
    const double e = fma(-(d * y), y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

// lambda_g = sym(alpha_g)^{-1} rho_g by Cholesky (Algorithm 1 line 7) for
// group g on one wave. Lane i holds row i of the symmetric part; step j takes
// row j of the Schur complement from lane j (readlane) as its column j (the
// complement stays symmetric up to rounding), and every lane subtracts
// L_ij / L_jj times it. Then lane c solves L L^T x = rho_:c by substitution
// against L in LDS. Lw: P * P + P doubles of LDS owned by the wave.
template <int P>
__device__ __forceinline__ void lambda_wave(const Plan& pl, const double* alpha, const double* rho, double* lam,
                                            float* lam32, DevState* st, int g, int lane, double* Lw) {
  constexpr int PP = P * P;
  const double* al = alpha + (int64_t)g * PP;
  const double* rh = rho + (int64_t)g * PP;
  const int i = lane < P ? lane : P - 1;
  double a[P], y[P];
  bool bad = false;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    a[c] = 0.5 * (al[i * P + c] + al[c * P + i]);
    y[c] = rh[c * P + i];  // column i of rho
    bad |= !isfinite(a[c]) || !isfinite(y[c]);
  }
  const double dg = al[i * P + i];
  bad = __any(bad);
  double rinv = 0.0;  // 1 / L_ii
  if (!bad) {
    // Step j scales column j of the Schur complement by 1 / sqrt(d) (lane j:
    // d / sqrt(d) = L_jj) and subtracts the outer product from the trailing
    // rows. Rows <= j also run the update, on entries above the diagonal
    // that are never read again.
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const double d = readlane_d(a[j], j);
      const double ajj = readlane_d(dg, j);
      if (!isfinite(d) || !(d > P * DBL_EPSILON * ajj) || !(ajj > 0.0)) {
        bad = true;
        break;
      }
      const double r = rsqrt_nr(d);
      a[j] *= r;                    // L_ij
      const double l2 = a[j] * r;   // L_ij / L_jj
#pragma unroll
      for (int c = j + 1; c < P; ++c) a[c] = fma(-l2, readlane_d(a[c], j), a[c]);  // - L_ij L_cj
      rinv = lane == j ? r : rinv;
    }
  }
  if (bad) {
    if (lane == 0) set_status(st, BCG_EBREAKDOWN);
    return;
  }
  wsync();  // the wave's previous use of Lw is complete
  if (lane < P) {
#pragma unroll
    for (int c = 0; c < P; ++c) Lw[lane * P + c] = a[c];
    Lw[PP + lane] = rinv;
  }
  wsync();
  if (lane < P) {  // lane = right-hand-side column
    const int c = lane;
    // The loads of step m are tied to the result of step m - 1 (an empty asm
    // with that input): without it the compiler issues every load of L
    // first and spills them.
#pragma unroll
    for (int m = 0; m < P; ++m) {  // L y = rho
      const double* Lm = Lw + after(m > 0 ? y[m - 1] : 0.0);
      y[m] *= Lm[PP + m];
#pragma unroll
      for (int r = m + 1; r < P; ++r) y[r] = fma(-Lm[r * P + m], y[m], y[r]);
    }
#pragma unroll
    for (int m = P - 1; m >= 0; --m) {  // L^T x = y
      const double* Lm = Lw + after(y[m < P - 1 ? m + 1 : m]);
      y[m] *= Lm[PP + m];
#pragma unroll
      for (int r = 0; r < m; ++r) y[r] = fma(-Lm[m * P + r], y[m], y[r]);
    }
#pragma unroll
    for (int r = 0; r < P; ++r) {
      lam[(int64_t)g * PP + r * P + c] = y[r];
      lam32[(int64_t)g * PP + r * P + c] = static_cast<float>(y[r]);
    }
  }
}

// Stop rule after the residual update (line 12): the largest column ratio
// ||R_j|| / r0_j against tol, then the iteration cap; a non-finite ratio is
// a breakdown. One whole wave evaluates it (every wave that calls it reaches
// the same decision); `lead` records the state, `wr` the ratios. Returns true
// when this iteration is the last (beta is not needed).
__device__ __forceinline__ bool stop_rule_wave(const Plan& pl, const double* red_new, const double* __restrict__ r0,
                                               double* __restrict__ ratios, DevState* st, double tol, int it,
                                               int maxit, int lane, bool lead, bool wr) {
  const int k = pl.k;
  double mx = 0.0;
  bool badr = false;
  for (int j = lane; j < k; j += 64) {
    const double c = red_new[pl.E + j];
    const double rr = r0[j];
    const double ratio = (rr == 0.0) ? 0.0 : sqrt(c) / rr;
    if (!isfinite(ratio))
      badr = true;
    else
      mx = fmax(mx, ratio);
    if (wr) ratios[j] = ratio;
  }
  for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off));
  badr = __any(badr);
  if (lead) {
    st->iter = it;
    st->max_ratio = badr ? NAN : mx;
  }
  if (badr) {
    if (lead) set_last(st, BCG_EBREAKDOWN);
    return true;
  }
  if (mx <= tol) {
    if (lead) set_last(st, BCG_OK);
    return true;
  }
  if (it >= maxit) {
    if (lead) set_last(st, BCG_NOT_CONVERGED);
    return true;
  }
  return false;
}

// beta_g = rho_g^{-1} rho_new_g by LU with partial pivoting (line 12) for
// group g on one wave: the largest magnitude in the pivot column, the first
// in the current row order on ties. Lane i holds row i of rho and tracks the
// position of that row; the pivot search runs over the 16-lane DPP rows
// holding candidates (two for p = 32), the pivot row is broadcast by
// readlane, and lane i stores its multiplier of every step in LDS. Then lane
// c takes column c of rho_new in pivot order and solves L z = y (unit lower,
// the multipliers in the same order of operations as an elimination of
// [rho | rho_new]) and U x = z against L and U in LDS. LDS owned by the wave:
// U (P * P by position, then the P reciprocal pivots), Lw (P * P by
// physical row and step), perm (P: physical row at each position).
template <int P>
__device__ __forceinline__ void beta_wave(const Plan& pl, const double* red_new, const double* rho_old, double* beta,
                                          float* beta32, DevState* st, int g, int lane, double* U, double* Lw,
                                          int* perm) {
  static_assert(P <= 32, "two DPP rows hold the candidate rows");
  constexpr int PP = P * P;
  const int i = lane < P ? lane : P - 1;
  double m[P];
  bool fail = false;
#pragma unroll
  for (int c = 0; c < P; ++c) {
    m[c] = rho_old[(int64_t)g * PP + i * P + c];
    fail |= !isfinite(m[c]);
  }
  fail = __any(fail);
  int pos = lane;     // current position of the row this lane holds
  double rpiv = 0.0;  // 1 / pivot of the step that placed this row
  wsync();            // the wave's previous use of its LDS is complete
  if (!fail) {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const bool cand = lane < P && pos >= j;
      const double v = cand ? fabs(m[j]) : -1.0;
      const double vr = row16_max(v);
      const double vmax = P > 16 ? fmax(readlane_d(vr, 0), readlane_d(vr, 16)) : readlane_d(vr, 0);
      if (!(vmax > 0.0)) {
        fail = true;
        break;
      }
      const int key = (cand && v == vmax) ? pos : P;
      const int kr = row16_min(key);
      const int kmin = P > 16 ? min(__builtin_amdgcn_readlane(kr, 0), __builtin_amdgcn_readlane(kr, 16))
                              : __builtin_amdgcn_readlane(kr, 0);
      const int piv = __ffsll(static_cast<long long>(__ballot(lane < P && pos == kmin))) - 1;
      const int at_j = __ffsll(static_cast<long long>(__ballot(lane < P && pos == j))) - 1;
      if (lane == piv)
        pos = j;
      else if (lane == at_j)
        pos = kmin;
      const double r = 1.0 / readlane_d(m[j], piv);
      rpiv = lane == piv ? r : rpiv;
      // rows at or above the pivot position subtract 0 * (pivot row)
      const double l = (lane < P && pos > j) ? m[j] * r : 0.0;
#pragma unroll
      for (int c = j + 1; c < P; ++c) m[c] = fma(-l, readlane_d(m[c], piv), m[c]);
      if (lane < P) Lw[lane * P + j] = l;
    }
  }
  if (fail) {
    if (lane == 0) set_last(st, BCG_EBREAKDOWN);
    return;
  }
  if (lane < P) {
#pragma unroll
    for (int c = 0; c < P; ++c) U[pos * P + c] = m[c];
    U[PP + pos] = rpiv;
    perm[pos] = lane;
  }
  wsync();
  if (lane < P) {
    const int c = lane;
    int rowq[P];
    double x[P];
#pragma unroll
    for (int q = 0; q < P; ++q) rowq[q] = perm[q];
#pragma unroll
    for (int q = 0; q < P; ++q) x[q] = red_new[(int64_t)g * PP + rowq[q] * P + c];
    // L z = y: the loads of step t are tied to the result of step t - 1
#pragma unroll
    for (int t = 0; t < P - 1; ++t) {
      const double* Lt = Lw + t + after(t > 0 ? x[t - 1] : 0.0);
#pragma unroll
      for (int q = t + 1; q < P; ++q) x[q] = fma(-Lt[rowq[q] * P], x[t], x[q]);
    }
#pragma unroll
    for (int mm = P - 1; mm >= 0; --mm) {  // U x = z, loads tied to the previous step
      const double* Um = U + after(x[mm < P - 1 ? mm + 1 : mm]);
      x[mm] *= Um[PP + mm];
#pragma unroll
      for (int r = 0; r < mm; ++r) x[r] = fma(-Um[r * P + mm], x[mm], x[r]);
    }
#pragma unroll
    for (int r = 0; r < P; ++r) {
      beta[(int64_t)g * PP + r * P + c] = x[r];
      beta32[(int64_t)g * PP + r * P + c] = static_cast<float>(x[r]);
    }
  }
}

// The fused reduce-and-solve launches: 8 entries per block, 512 threads
// (the solves get the register budget of 2 waves per SIMD).
constexpr int kFuseEntries = 8;
constexpr int kFuseSlots = 64;
constexpr int kFuseThreads = kFuseSlots * kFuseEntries;
constexpr int kFuseWaves = kFuseThreads / 64;
// waves of the last workgroup that solve (one group each); p = 32 keeps the
// LDS of its factors to two waves
template <int P>
constexpr int solve_waves() {
  return P > 16 ? 2 : kFuseWaves;
}

// Lines 6-7 in one launch: blocks [0, nb) sum alpha over a_rows partial
// rows, blocks [nb, 2 nb) (r_rows > 0) rho over r_rows; for P > 0 the block
// that finishes last solves for lambda, one wave per group. After the final
// iteration it only sets `done`.
template <int P>
__global__ __launch_bounds__(kFuseThreads) void k_reduce_lambda(Plan pl, const double* __restrict__ partA,
                                                                int a_rows, const double* __restrict__ partR,
                                                                int r_rows, double* alpha, double* rho, double* lam,
                                                                float* lam32, DevState* st) {
  if (stopped(st)) return;
  if (*reinterpret_cast<const volatile int*>(&st->last)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *reinterpret_cast<volatile int*>(&st->done) = 1;
    return;
  }
  __shared__ double sh[kFuseSlots][kFuseEntries];
  const int nb = (pl.E + kFuseEntries - 1) / kFuseEntries;
  if (static_cast<int>(blockIdx.x) < nb)
    reduce_entries<kFuseEntries, kFuseSlots>(partA, alpha, pl.E, pl.W, 0, a_rows, blockIdx.x, sh);
  else
    reduce_entries<kFuseEntries, kFuseSlots>(partR, rho, pl.E, pl.W, 0, r_rows, blockIdx.x - nb, sh);
  if constexpr (P > 0) {
    if (!last_workgroup(st)) return;
    constexpr int SW = solve_waves<P>();
    __shared__ double Ls[SW][P * P + P];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave >= SW) return;
    for (int g = wave; g < pl.qo; g += SW) lambda_wave<P>(pl, alpha, rho, lam, lam32, st, opaque(g), lane, Ls[wave]);
  }
}

// Line 11 sums (<<R, R>> and the column norms) over `rows` partial rows,
// then in the block that finishes last the stop rule and beta (line 12).
template <int P>
__global__ __launch_bounds__(kFuseThreads) void k_reduce_beta(Plan pl, const double* __restrict__ partN, int rows,
                                                              double* red_new, const double* __restrict__ r0,
                                                              const double* __restrict__ rho_old,
                                                              double* __restrict__ beta, float* __restrict__ beta32,
                                                              double* __restrict__ ratios, DevState* st, double tol,
                                                              int it, int maxit) {
  if (stopped(st)) return;
  __shared__ double sh[kFuseSlots][kFuseEntries];
  reduce_entries<kFuseEntries, kFuseSlots>(partN, red_new, pl.W, pl.W, 0, rows, blockIdx.x, sh);
  if (!last_workgroup(st)) return;
  constexpr int SW = solve_waves<P>();
  __shared__ double Us[SW][P * P + P];
  __shared__ double Ls[SW][P * P];
  __shared__ int Pm[SW][P];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (wave >= SW) return;
  if (stop_rule_wave(pl, red_new, r0, ratios, st, tol, it, maxit, lane, threadIdx.x == 0, wave == 0)) return;
  for (int g = wave; g < pl.qo; g += SW)
    beta_wave<P>(pl, red_new, rho_old, beta, beta32, st, opaque(g), lane, Us[wave], Ls[wave], Pm[wave]);
}

// ---- workgroup Gauss-Jordan for p x p groups with 16 < p <= 64 (and the
// odd sizes below 16): [A | B] (p x 2p) in LDS; per step the pivot row and
// column are copied aside and every thread updates its entries (thread t:
// column t mod 2p of every (256 / 2p)-th row). Without row exchanges (line 7)
// the pivots are the diagonals of the successive Schur complements, tested
// with the Cholesky rule; with partial pivoting (line 12) the pivots and
// their order are those of LU with partial pivoting.
constexpr int kGJMaxP = 64;

struct GJShared {
  double M[kGJMaxP * 2 * kGJMaxP];
  double colb[kGJMaxP];
  double rowb[2 * kGJMaxP];
  double dg0[kGJMaxP];
  int flag[2];
};

// Returns true (workgroup-uniform) on breakdown. NS >= the rows a thread
// updates (p / (256 / 2p), rounded up): its entries are loaded before any is
// stored, so the loads of a step are in flight together.
template <int NS>
__device__ __forceinline__ bool wg_gauss_jordan(GJShared& S, int p, bool cholesky_rule, bool pivoting) {
  const int tid = threadIdx.x, w2 = 2 * p;
  const int rpp = kBlock / w2;                 // rows per pass
  const int c = tid % w2, r0 = tid / w2;      // this thread's column, first row
  const bool act = r0 < rpp;
  for (int j = 0; j < p; ++j) {
    if (pivoting) {
      if (tid < 64) {  // one wave: rows j..p-1 of column j
        const int r = tid;
        const bool cand = r >= j && r < p;
        double v = cand ? fabs(S.M[r * w2 + j]) : -1.0;
        const bool nan = __any(cand && !(v == v));
        int key = r;
        for (int off = 32; off > 0; off >>= 1) {
          const double ov = __shfl_xor(v, off);
          const int ok = __shfl_xor(key, off);
          if (ov > v || (ov == v && ok < key)) {
            v = ov;
            key = ok;
          }
        }
        if (tid == 0) {
          S.flag[0] = (nan || !(v > 0.0)) ? 1 : 0;
          S.flag[1] = key;
        }
      }
      __syncthreads();
      if (S.flag[0]) return true;
      const int piv = S.flag[1];
      if (piv != j) {
        for (int cc = tid; cc < w2; cc += kBlock) {
          const double a = S.M[j * w2 + cc];
          S.M[j * w2 + cc] = S.M[piv * w2 + cc];
          S.M[piv * w2 + cc] = a;
        }
        __syncthreads();
      }
    }
    for (int cc = tid; cc < w2; cc += kBlock) S.rowb[cc] = S.M[j * w2 + cc];
    for (int r = tid; r < p; r += kBlock) S.colb[r] = S.M[r * w2 + j];
    __syncthreads();
    const double d = S.rowb[j];
    if (cholesky_rule) {
      const double ajj = S.dg0[j];
      if (!isfinite(d) || !(d > p * DBL_EPSILON * ajj) || !(ajj > 0.0)) return true;
    }
    const double inv = 1.0 / d;
    if (act) {
      const double rc = S.rowb[c];
      double t[NS];
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int r = r0 + rpp * u;
        t[u] = r < p ? S.M[r * w2 + c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < NS; ++u) {
        const int r = r0 + rpp * u;
        if (r < p) S.M[r * w2 + c] = r == j ? rc * inv : t[u] - S.colb[r] * inv * rc;
      }
    }
    __syncthreads();
  }
  return false;
}

// lambda_g = sym(alpha_g)^{-1} rho_g (Algorithm 1 line 7), one workgroup per group.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_solve_lambda_gj(Plan pl, const double* __restrict__ alpha,
                                                            const double* __restrict__ rho, double* __restrict__ lam,
                                                            float* __restrict__ lam32, DevState* st) {
  if (stopped(st)) return;
  __shared__ GJShared S;
  const int tid = threadIdx.x, g = blockIdx.x, p = pl.p, pp = p * p, w2 = 2 * p;
  const double* al = alpha + (int64_t)g * pp;
  const double* rh = rho + (int64_t)g * pp;
  int bad = 0;
  for (int e = tid; e < p * w2; e += kBlock) {
    const int r = e / w2, c = e - r * w2;
    const double v = c < p ? 0.5 * (al[r * p + c] + al[c * p + r]) : rh[r * p + (c - p)];
    S.M[e] = v;
    if (!isfinite(v)) bad = 1;
    if (c == r) S.dg0[r] = v;
  }
  if (__syncthreads_or(bad) || wg_gauss_jordan<NS>(S, p, true, false)) {
    if (tid == 0) set_status(st, BCG_EBREAKDOWN);
    return;
  }
  for (int e = tid; e < pp; e += kBlock) {
    const int r = e / p, c = e - r * p;
    const double v = S.M[r * w2 + p + c];
    lam[(int64_t)g * pp + e] = v;
    lam32[(int64_t)g * pp + e] = static_cast<float>(v);
  }
}

// Stop rule, then beta_g = rho_g^{-1} rho_new_g (Algorithm 1 lines 9-12), one
// workgroup per group; every workgroup evaluates the rule, workgroup 0 records it.
template <int NS>
__global__ __launch_bounds__(kBlock) void k_conv_beta_gj(Plan pl, const double* __restrict__ red_new,
                                                         const double* __restrict__ r0,
                                                         const double* __restrict__ rho_old, double* __restrict__ beta,
                                                         float* __restrict__ beta32, double* __restrict__ ratios,
                                                         DevState* st, double tol, int it, int maxit) {
  if (stopped(st)) return;
  __shared__ GJShared S;
  __shared__ double smax[kBlock];
  __shared__ int sbad[kBlock];
  const int tid = threadIdx.x, k = pl.k, p = pl.p, pp = p * p, w2 = 2 * p, g = blockIdx.x;
  double m = 0.0;
  int bad = 0;
  for (int j = tid; j < k; j += kBlock) {
    const double cn = red_new[pl.E + j];
    const double rr = r0[j];
    const double ratio = (rr == 0.0) ? 0.0 : sqrt(cn) / rr;
    if (!isfinite(ratio))
      bad = 1;
    else
      m = fmax(m, ratio);
    if (g == 0) ratios[j] = ratio;
  }
  smax[tid] = m;
  sbad[tid] = bad;
  __syncthreads();
  for (int s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      smax[tid] = fmax(smax[tid], smax[tid + s]);
      sbad[tid] |= sbad[tid + s];
    }
    __syncthreads();
  }
  const bool lead = g == 0 && tid == 0;
  if (lead) {
    st->iter = it;
    st->max_ratio = sbad[0] ? NAN : smax[0];
  }
  if (sbad[0]) {
    if (lead) set_last(st, BCG_EBREAKDOWN);
    return;
  }
  if (smax[0] <= tol) {
    if (lead) set_last(st, BCG_OK);
    return;
  }
  if (it >= maxit) {
    if (lead) set_last(st, BCG_NOT_CONVERGED);
    return;
  }
  const double* ro = rho_old + (int64_t)g * pp;
  const double* rn = red_new + (int64_t)g * pp;
  bad = 0;
  for (int e = tid; e < p * w2; e += kBlock) {
    const int r = e / w2, c = e - r * w2;
    const double v = c < p ? ro[r * p + c] : rn[r * p + (c - p)];
    S.M[e] = v;
    if (c < p && !isfinite(v)) bad = 1;
  }
  if (__syncthreads_or(bad) || wg_gauss_jordan<NS>(S, p, false, true)) {
    if (tid == 0) set_last(st, BCG_EBREAKDOWN);
    return;
  }
  for (int e = tid; e < pp; e += kBlock) {
    const int r = e / p, c = e - r * p;
    const double v = S.M[r * w2 + p + c];
    beta[(int64_t)g * pp + e] = v;
    beta32[(int64_t)g * pp + e] = static_cast<float>(v);
  }
}

// rows per thread of the workgroup Gauss-Jordan for p, rounded up to a power of two
template <typename F>
void dispatch_gj_slots(int p, F&& f) {
  const int rpp = kBlock / (2 * p), need = (p + rpp - 1) / rpp;
  if (need <= 2)
    f(std::integral_constant<int, 2>());
  else if (need <= 4)
    f(std::integral_constant<int, 4>());
  else if (need <= 8)
    f(std::integral_constant<int, 8>());
  else if (need <= 16)
    f(std::integral_constant<int, 16>());
  else
    f(std::integral_constant<int, 32>());
}

template <typename F>
bool dispatch_small_p(int p, F&& f) {
  switch (p) {
    case 2: f(std::integral_constant<int, 2>()); return true;
    case 4: f(std::integral_constant<int, 4>()); return true;
    case 8: f(std::integral_constant<int, 8>()); return true;
    case 16: f(std::integral_constant<int, 16>()); return true;
    case 32: f(std::integral_constant<int, 32>()); return true;
    default: return false;
  }
}

__global__ __launch_bounds__(kBlock) void k_axpy_scaled(int64_t count, double* __restrict__ X,
                                                        const float* __restrict__ D, const double* __restrict__ scale) {
  const double s = *scale;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < count; e += (int64_t)gridDim.x * kBlock)
    X[e] += s * static_cast<double>(D[e]);
}

__global__ __launch_bounds__(kBlock) void k_cast_values(int64_t nnz, const double* __restrict__ v,
                                                        float* __restrict__ v32) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * kBlock)
    v32[e] = static_cast<float>(v[e]);
}

__global__ __launch_bounds__(kBlock) void k_sell_values(int64_t slots, const int32_t* __restrict__ map,
                                                        const double* __restrict__ v, const float* __restrict__ v32,
                                                        double* __restrict__ sv, float* __restrict__ sv32) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < slots; e += (int64_t)gridDim.x * kBlock) {
    const int32_t m = map[e];
    sv[e] = m >= 0 ? v[m] : 0.0;
    sv32[e] = m >= 0 ? v32[m] : 0.f;
  }
}

// out[e] = alpha * <Y[row(e), :], X[col(e), :]>; L lanes per row.
__global__ __launch_bounds__(kBlock) void k_sampled_outer(int64_t n, int k, int L, const int32_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ colind,
                                                          const double* __restrict__ Y, const double* __restrict__ X,
                                                          double alpha, double* __restrict__ out) {
  const int64_t gt = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  const int64_t row = gt / L;
  const int lane = static_cast<int>(gt % L);
  if (row >= n) return;  // whole L-lane groups leave together (L divides 64)
  const double* yr = Y + row * k;
  const int j1 = rowptr[row + 1];
  for (int j = rowptr[row]; j < j1; ++j) {
    const double* xr = X + (int64_t)colind[j] * k;
    double s = 0.0;
    for (int c = lane; c < k; c += L) s = fma(yr[c], xr[c], s);
    for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
    if (lane == 0) out[j] = alpha * s;
  }
}

// ------------------------------------------------------------------------
// Template dispatch on the accumulation shape
// ------------------------------------------------------------------------
template <typename F>
void dispatch_shape(const Plan& pl, F&& f) {
  if (pl.rb == 2) {
    if (pl.EB <= kBlock)
      f(std::integral_constant<int, 2>(), std::integral_constant<int, 1>());
    else
      f(std::integral_constant<int, 2>(), std::integral_constant<int, kNabMax>());
  } else {
    if (pl.EB <= kBlock)
      f(std::integral_constant<int, 1>(), std::integral_constant<int, 1>());
    else
      f(std::integral_constant<int, 1>(), std::integral_constant<int, kNabMax>());
  }
}

// flag = 1 if order is not a permutation of 0..n-1: an entry outside [0, n),
// or a row taken twice (seen: n zeroed counters).
__global__ __launch_bounds__(kBlock) void k_check_perm(const int32_t* __restrict__ order, int64_t n,
                                                       int* __restrict__ seen, int* __restrict__ flag) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < n; e += (int64_t)gridDim.x * kBlock) {
    const int32_t v = order[e];
    if (v < 0 || v >= n || atomicAdd(seen + v, 1) != 0) *reinterpret_cast<volatile int*>(flag) = 1;
  }
}

// flag = 1 unless the CSR arrays describe n rows of nnz entries: rowptr[0] =
// 0, rowptr non-decreasing, rowptr[n] = nnz, every column in [0, n). Only
// rowptr[0..n] and colind[0..nnz) are read, so a malformed matrix is
// rejected before any kernel follows its row ranges.
__global__ __launch_bounds__(kBlock) void k_check_csr(const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind, int64_t n, int64_t nnz,
                                                      int* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i <= n; i += stride) {
    const int32_t a = rowptr[i];
    if (i == 0 && a != 0) bad = true;
    if (i == n && a != nnz) bad = true;
    if (i < n && rowptr[i + 1] < a) bad = true;
  }
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < nnz; e += stride) {
    const int32_t c = colind[e];
    if (c < 0 || c >= n) bad = true;
  }
  if (bad) *reinterpret_cast<volatile int*>(flag) = 1;
}

// Jacobi preconditioner M = diag(A): s_i = 1 / sqrt(a_ii) (duplicate
// diagonal entries summed). flag = 1 when a row has no diagonal entry or
// a_ii is not positive and finite (s_i = 1 there).
__global__ __launch_bounds__(kBlock) void k_jacobi_scale(int64_t n, const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colind,
                                                         const double* __restrict__ vals, double* __restrict__ dscale,
                                                         int* __restrict__ flag) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    double d = 0.0;
    bool found = false;
    const int j1 = rowptr[i + 1];
    for (int j = rowptr[i]; j < j1; ++j)
      if (colind[j] == i) {
        d += vals[j];
        found = true;
      }
    const bool ok = found && d > 0.0 && isfinite(d);
    if (!ok) *reinterpret_cast<volatile int*>(flag) = 1;
    dscale[i] = ok ? 1.0 / sqrt(d) : 1.0;
  }
}

// Values of D^{-1/2} A D^{-1/2}: s_row * a * s_col, in FP64 and FP32.
__global__ __launch_bounds__(kBlock) void k_scale_values(int64_t n, const int32_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colind,
                                                         const double* __restrict__ vals,
                                                         const double* __restrict__ dscale, double* __restrict__ vs,
                                                         float* __restrict__ vs32) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    const double si = dscale[i];
    const int j1 = rowptr[i + 1];
    for (int j = rowptr[i]; j < j1; ++j) {
      const double v = si * vals[j] * dscale[colind[j]];
      vs[j] = v;
      vs32[j] = static_cast<float>(v);
    }
  }
}

// dst = D^{-1/2} src (divide = 0) or D^{1/2} src (divide = 1), row-major
// n x k; dst may be src.
__global__ __launch_bounds__(kBlock) void k_scale_rows(int64_t n, int k, const double* src,
                                                       const double* __restrict__ dscale, double* dst, int divide) {
  const int64_t count = n * k;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < count; e += (int64_t)gridDim.x * kBlock) {
    const double si = dscale[e / k];
    dst[e] = divide ? src[e] / si : src[e] * si;
  }
}

}  // namespace

void launch_jacobi_scale(int64_t n, const int32_t* rowptr, const int32_t* colind, const double* vals, double* dscale,
                         int* flag, hipStream_t s) {
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  hipLaunchKernelGGL(k_jacobi_scale, dim3(grid), dim3(kBlock), 0, s, n, rowptr, colind, vals, dscale, flag);
}

void launch_scale_values(int64_t n, const int32_t* rowptr, const int32_t* colind, const double* vals,
                         const double* dscale, double* vs, float* vs32, hipStream_t s) {
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  hipLaunchKernelGGL(k_scale_values, dim3(grid), dim3(kBlock), 0, s, n, rowptr, colind, vals, dscale, vs, vs32);
}

void launch_scale_rows(int64_t n, int k, const double* src, const double* dscale, double* dst, int divide,
                       hipStream_t s) {
  const int64_t blocks = (n * k + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(blocks < 8192 ? (blocks > 0 ? blocks : 1) : 8192);
  hipLaunchKernelGGL(k_scale_rows, dim3(grid), dim3(kBlock), 0, s, n, k, src, dscale, dst, divide);
}

void launch_check_perm(const int32_t* order, int64_t n, int* seen, int* flag, hipStream_t s) {
  const int64_t blocks = (n + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  hipLaunchKernelGGL(k_check_perm, dim3(grid), dim3(kBlock), 0, s, order, n, seen, flag);
}

void launch_check_csr(const int32_t* rowptr, const int32_t* colind, int64_t n, int64_t nnz, int* flag,
                      hipStream_t s) {
  const int64_t m = std::max<int64_t>(n + 1, nnz), blocks = (m + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  hipLaunchKernelGGL(k_check_csr, dim3(grid), dim3(kBlock), 0, s, rowptr, colind, n, nnz, flag);
}

Plan make_plan(int64_t n, int64_t nnz, int k, int p, int global, int dec) {
  Plan pl{};
  pl.n = n;
  pl.nnz = nnz;
  pl.k = k;
  pl.p = p;
  pl.q = k / p;
  pl.global = global;
  pl.dec = dec;
  pl.qo = global ? 1 : pl.q;
  pl.E = pl.qo * p * p;
  pl.W = pl.E + k;
  pl.rb = (p % 2 == 0) ? 2 : 1;
  pl.pb = p / pl.rb;
  pl.EB = pl.qo * pl.pb * pl.pb;
  if (pl.EB <= kBlock) {
    pl.S = kBlock / pl.EB;
    pl.nab = 1;
  } else {
    pl.S = 1;
    pl.nab = (pl.EB + kBlock - 1) / kBlock;
  }
  pl.fused = pl.nab <= kNabMax;
  pl.TR = kTileElems / k > 0 ? kTileElems / k : 1;
  pl.ntiles = (n + pl.TR - 1) / pl.TR;
  // rows per wave step of the fast kernels (k/2 lanes per row), 4 waves per group
  const int64_t rw = k >= 2 && k <= 128 ? 128 / k : 1;
  const int64_t fwg = ((n + rw - 1) / rw + 3) / 4;
  int64_t nwg = pl.ntiles < fwg ? pl.ntiles : fwg;
  if (nwg > kMaxWG) nwg = kMaxWG;
  pl.nwg = static_cast<int>(nwg < 1 ? 1 : nwg);
  pl.fast = fast_supported(pl);
  pl.mfma = mfma_width(nnz, k, p);
  pl.sp_w = pl.mfma ? mfma_sp_width(k, pl.mfma, p) : 0;
  if (pl.mfma) {
    pl.nwg = mfma_grid(n, k, pl.mfma);
    mfma_sp_grid(pl);
  }
  return pl;
}

void launch_residual(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const double* vals,
                     const double* B, const double* X, double* R, double* P, double* part, int with_p,
                     hipStream_t s) {
  // the k-specialised gather kernel where the plan has one and every block
  // vector is 16-byte aligned (it moves two columns per lane)
  const uintptr_t al = reinterpret_cast<uintptr_t>(B) | reinterpret_cast<uintptr_t>(X) |
                       reinterpret_cast<uintptr_t>(R) | reinterpret_cast<uintptr_t>(with_p ? P : R);
  if (pl.fast && al % 16 == 0 && (!with_p || pl.fused) &&
      launch_residual_fast(pl, rowptr, colind, vals, B, X, R, P, part, with_p, s))
    return;
  dispatch_shape(pl, [&](auto RB, auto NAB) {
    hipLaunchKernelGGL((k_residual<decltype(RB)::value, decltype(NAB)::value>), dim3(pl.nwg), dim3(kBlock), 0, s, pl, rowptr, colind, vals, B, X,
                       R, P, part, with_p);
  });
}

void launch_cast_init(const Plan& pl, const double* R64, const double* norms, float* R32, float* P32, float* D32,
                      double* scale, double* part, hipStream_t s, double pfac) {
  // the k-specialised kernel moves two columns per lane: every block 8-byte
  // (FP32) or 16-byte (FP64) aligned
  const uintptr_t al = reinterpret_cast<uintptr_t>(R32) | reinterpret_cast<uintptr_t>(P32) |
                       reinterpret_cast<uintptr_t>(D32);
  if (pl.fast && pl.fused && al % 8 == 0 && reinterpret_cast<uintptr_t>(R64) % 16 == 0 &&
      launch_cast_init_fast(pl, R64, norms, R32, P32, D32, scale, part, s, pfac))
    return;
  dispatch_shape(pl, [&](auto RB, auto NAB) {
    hipLaunchKernelGGL((k_cast_init<decltype(RB)::value, decltype(NAB)::value>), dim3(pl.nwg), dim3(kBlock), 0, s, pl, R64, norms, R32, P32, D32,
                       scale, part, pfac);
  });
}

__global__ __launch_bounds__(kBlock) void k_scale_vec(double* __restrict__ x, int64_t count, double c) {
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < count; e += (int64_t)gridDim.x * kBlock) x[e] *= c;
}

void launch_scale_vec(double* x, int64_t count, double c, hipStream_t s) {
  const int64_t blocks = (count + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(blocks < 1024 ? (blocks > 0 ? blocks : 1) : 1024);
  hipLaunchKernelGGL(k_scale_vec, dim3(grid), dim3(kBlock), 0, s, x, count, c);
}

template <typename T>
void launch_spmm_product(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const T* vals, const T* P,
                         T* Q, double* part, const DevState* st, hipStream_t s) {
  dispatch_shape(pl, [&](auto RB, auto NAB) {
    hipLaunchKernelGGL((k_spmm_product<T, decltype(RB)::value, decltype(NAB)::value>), dim3(pl.nwg), dim3(kBlock), 0, s, pl, rowptr, colind, vals,
                       P, Q, part, st);
  });
}

template <typename T>
void launch_update_r(const Plan& pl, T* R, const T* Q, const T* lam, double* part, const DevState* st,
                     hipStream_t s) {
  dispatch_shape(pl, [&](auto RB, auto NAB) {
    hipLaunchKernelGGL((k_update_r<T, decltype(RB)::value, decltype(NAB)::value>), dim3(pl.nwg), dim3(kBlock), 0, s,
                       pl, R, Q, lam, part, st);
  });
}

template <typename T>
void launch_update_xp(const Plan& pl, T* X, T* P, const T* R, const T* lam, const T* beta, double* part,
                      const DevState* st, hipStream_t s) {
  dispatch_shape(pl, [&](auto RB, auto NAB) {
    hipLaunchKernelGGL((k_update_xp<T, decltype(RB)::value, decltype(NAB)::value>), dim3(pl.nwg), dim3(kBlock), 0,
                       s, pl, X, P, R, lam, beta, part, st);
  });
}

template <typename T>
void launch_product(const Plan& pl, const T* X, const T* Y, double* part, const DevState* st, hipStream_t s) {
  const int chunk = kNabMax * kBlock;
  for (int off = 0; off < pl.EB; off += chunk) {
    if (pl.rb == 2)
      hipLaunchKernelGGL((k_product<T, 2, kNabMax>), dim3(pl.nwg), dim3(kBlock), 0, s, pl, X, Y, part, st, off);
    else
      hipLaunchKernelGGL((k_product<T, 1, kNabMax>), dim3(pl.nwg), dim3(kBlock), 0, s, pl, X, Y, part, st, off);
  }
}

void launch_reduce(const Plan& pl, const double* part, double* out, int width, DevState* st, hipStream_t s, int rows,
                   double* scratch) {
  if (rows < 0) rows = pl.nwg;
  if (rows > kRedSplitRows && scratch != nullptr) {
    hipLaunchKernelGGL(k_reduce_rows, dim3((width + kRowsEPB - 1) / kRowsEPB, kRedSplits), dim3(kRowsThreads), 0, s,
                       part, scratch, width, pl.W, rows, st);
    part = scratch;
    rows = kRedSplits;
  }
  hipLaunchKernelGGL(k_reduce, dim3((width + 15) / 16), dim3(kRedThreads), 0, s, part, out, width, pl.W, rows, st);
}

bool register_solve(int p) { return p == 2 || p == 4 || p == 8 || p == 16 || p == 32; }

void launch_reduce_lambda(const Plan& pl, const double* partA, int a_rows, double* scratch, const double* partR,
                          int r_rows, double* alpha, double* rho, double* lam, float* lam32, double* ws, DevState* st,
                          hipStream_t s) {
  if (a_rows > kRedSplitRows && scratch != nullptr) {
    hipLaunchKernelGGL(k_reduce_rows, dim3((pl.E + kRowsEPB - 1) / kRowsEPB, kRedSplits), dim3(kRowsThreads), 0, s,
                       partA, scratch, pl.E, pl.W, a_rows, st);
    partA = scratch;
    a_rows = kRedSplits;
  }
  const int nb = (pl.E + kFuseEntries - 1) / kFuseEntries;
  const dim3 grid(r_rows > 0 ? 2 * nb : nb);
  if (dispatch_small_p(pl.p, [&](auto Pc) {
        hipLaunchKernelGGL((k_reduce_lambda<decltype(Pc)::value>), grid, dim3(kFuseThreads), 0, s, pl, partA, a_rows,
                           partR, r_rows, alpha, rho, lam, lam32, st);
      }))
    return;
  hipLaunchKernelGGL((k_reduce_lambda<0>), grid, dim3(kFuseThreads), 0, s, pl, partA, a_rows, partR, r_rows, alpha,
                     rho, lam, lam32, st);
  launch_solve_lambda(pl, alpha, rho, lam, lam32, ws, st, s);
}

void launch_reduce_beta(const Plan& pl, const double* partN, int rows, double* red_new, const double* r0,
                        const double* rho_old, double* beta, float* beta32, double* ws, double* ratios, DevState* st,
                        double tol, int it, int maxit, hipStream_t s) {
  if (dispatch_small_p(pl.p, [&](auto Pc) {
        hipLaunchKernelGGL((k_reduce_beta<decltype(Pc)::value>), dim3((pl.W + kFuseEntries - 1) / kFuseEntries),
                           dim3(kFuseThreads), 0, s, pl, partN, rows, red_new, r0, rho_old, beta, beta32, ratios, st,
                           tol, it, maxit);
      }))
    return;
  launch_reduce(pl, partN, red_new, pl.W, st, s, rows);
  launch_conv_beta(pl, red_new, r0, rho_old, beta, beta32, ws, ratios, st, tol, it, maxit, s);
}

void launch_solve_lambda(const Plan& pl, const double* alpha, const double* rho, double* lam, float* lam32,
                         double* ws, DevState* st, hipStream_t s) {
  if (pl.p > 1 && pl.p <= kGJMaxP) {
    dispatch_gj_slots(pl.p, [&](auto Nc) {
      hipLaunchKernelGGL((k_solve_lambda_gj<decltype(Nc)::value>), dim3(pl.qo), dim3(kBlock), 0, s, pl, alpha, rho,
                         lam, lam32, st);
    });
    return;
  }
  const int grid = pl.p == 1 ? 1 : pl.qo;
  hipLaunchKernelGGL(k_solve_lambda, dim3(grid), dim3(kBlock), 0, s, pl, alpha, rho, lam, lam32, ws, st);
}

void launch_conv_beta(const Plan& pl, const double* red_new, const double* r0, const double* rho_old, double* beta,
                      float* beta32, double* ws, double* ratios, DevState* st, double tol, int it, int maxit,
                      hipStream_t s) {
  if (pl.p > 1 && pl.p <= kGJMaxP) {
    dispatch_gj_slots(pl.p, [&](auto Nc) {
      hipLaunchKernelGGL((k_conv_beta_gj<decltype(Nc)::value>), dim3(pl.qo), dim3(kBlock), 0, s, pl, red_new, r0,
                         rho_old, beta, beta32, ratios, st, tol, it, maxit);
    });
    return;
  }
  const int grid = pl.p == 1 ? 1 : pl.qo;
  hipLaunchKernelGGL(k_conv_beta, dim3(grid), dim3(kBlock), 0, s, pl, red_new, r0, rho_old, beta, beta32, ws, ratios,
                     st, tol, it, maxit);
}

void launch_axpy_scaled(int64_t count, double* X, const float* D, const double* scale, hipStream_t s) {
  const int64_t blocks = (count + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  hipLaunchKernelGGL(k_axpy_scaled, dim3(grid), dim3(kBlock), 0, s, count, X, D, scale);
}

void launch_cast_values(int64_t nnz, const double* v, float* v32, hipStream_t s) {
  const int64_t blocks = (nnz + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  hipLaunchKernelGGL(k_cast_values, dim3(grid), dim3(kBlock), 0, s, nnz, v, v32);
}

void launch_sell_values(int64_t slots, const int32_t* map, const double* v, const float* v32, double* sv,
                        float* sv32, hipStream_t s) {
  const int64_t blocks = (slots + kBlock - 1) / kBlock;
  const int grid = static_cast<int>(blocks < 4096 ? (blocks > 0 ? blocks : 1) : 4096);
  hipLaunchKernelGGL(k_sell_values, dim3(grid), dim3(kBlock), 0, s, slots, map, v, v32, sv, sv32);
}

void launch_sampled_outer(int64_t n, int k, const int32_t* rowptr, const int32_t* colind, const double* Y,
                          const double* X, double alpha, double* out, hipStream_t s) {
  int L = 1;
  while (L * 2 <= k && L * 2 <= 64) L *= 2;
  const int64_t threads = n * L;
  const int64_t grid = (threads + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_sampled_outer, dim3(static_cast<unsigned>(grid)), dim3(kBlock), 0, s, n, k, L, rowptr, colind,
                     Y, X, alpha, out);
}

template void launch_spmm_product<double>(const Plan&, const int32_t*, const int32_t*, const double*, const double*,
                                          double*, double*, const DevState*, hipStream_t);
template void launch_spmm_product<float>(const Plan&, const int32_t*, const int32_t*, const float*, const float*,
                                         float*, double*, const DevState*, hipStream_t);
template void launch_update_r<double>(const Plan&, double*, const double*, const double*, double*, const DevState*,
                                      hipStream_t);
template void launch_update_r<float>(const Plan&, float*, const float*, const float*, double*, const DevState*,
                                     hipStream_t);
template void launch_update_xp<double>(const Plan&, double*, double*, const double*, const double*, const double*,
                                       double*, const DevState*, hipStream_t);
template void launch_update_xp<float>(const Plan&, float*, float*, const float*, const float*, const float*, double*,
                                      const DevState*, hipStream_t);
template void launch_product<double>(const Plan&, const double*, const double*, double*, const DevState*,
                                     hipStream_t);
template void launch_product<float>(const Plan&, const float*, const float*, double*, const DevState*, hipStream_t);

}  // namespace bcg
