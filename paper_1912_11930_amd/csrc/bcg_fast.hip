// Row kernels of the block CG iteration specialised on k (compile time) and a
// block size p <= 16, for gfx950.
//
// Mapping: each row of the n x k block vectors is handled by G = k/2 lanes,
// each lane owning two adjacent columns (one 16-byte load per operand in
// FP64, 8 bytes in FP32), so a wave covers 64/G rows per step and waves
// stride over the rows. The coefficient blocks (lambda, beta) of a lane's two
// columns stay in registers for the whole kernel. Where a lane needs the other
// columns of its group (p > 2) it reads them from a wave-private LDS slab of
// the rows it just loaded, so the main loop has no workgroup barrier.
//
// Block products: lane (row i, columns b0, b0+1 of group g) accumulates
// sum_i X[i, g*p + a] * Y[i, b] for a < p over all of its rows, in FP64.
// After the row loop the partial sums are combined across the row slots of
// the wave (butterfly over lane bits) and across the four waves (fixed order)
// and written as one packed partial [qo][p][p] (+ column norms) per
// workgroup, the same layout as the generic kernels.
#include <cstdlib>
#include <type_traits>

#include "../../include/bcg.h"
#include "bcg_internal.h"

namespace bcg {

namespace {

template <typename T>
struct V2;
template <>
struct V2<double> {
  using type = double2;
};
template <>
struct V2<float> {
  using type = float2;
};

__device__ __forceinline__ bool fstopped(const DevState* st) {
  return st != nullptr && *reinterpret_cast<const volatile int*>(&st->done) != 0;
}

// Orders this wave's LDS writes before its later LDS reads.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int K, int P>
struct Geo {
  static constexpr int V = 2;            // columns per lane
  static constexpr int G = K / V;        // lanes per row
  static constexpr int RW = 64 / G;      // rows per wave step
  static constexpr int SLAB = RW * K;    // elements of one wave slab
  static constexpr int NEED_LDS = P > V; // group spans several lanes
  static_assert(K % V == 0 && G <= 64 && 64 % G == 0, "unsupported k");
  static_assert(P <= K && K % P == 0, "p must divide k");
};

// Row steps of this wave. Workgroups are dispatched to the 8 XCDs round
// robin (workgroup b on XCD b % 8), so with at least 8 workgroups XCD x is
// given the contiguous eighth x of the row steps: the neighbour rows a
// stencil row gathers are then mostly its own, and stay in its L2.
struct StepRange {
  int64_t first, end, stride;
};

__device__ __forceinline__ StepRange wave_steps(int64_t nsteps) {
  const int nwg = gridDim.x, b = blockIdx.x, wave = threadIdx.x >> 6;
  StepRange r;
  if (nwg < 8) {
    r.first = (int64_t)b * 4 + wave;
    r.end = nsteps;
    r.stride = (int64_t)nwg * 4;
    return r;
  }
  const int x = b & 7, lb = b >> 3;
  const int nx = (nwg - x + 7) >> 3;  // workgroups on XCD x
  const int64_t per = (nsteps + 7) / 8;
  const int64_t lo = min((int64_t)x * per, nsteps);
  r.first = lo + (int64_t)lb * 4 + wave;
  r.end = min(lo + per, nsteps);
  r.stride = (int64_t)nx * 4;
  return r;
}

// Per-lane partial block product and column norms.
template <int P>
struct LaneAcc {
  double a[2][P];
  double nrm[2];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int v = 0; v < 2; ++v) {
#pragma unroll
      for (int j = 0; j < P; ++j) a[v][j] = 0.0;
      nrm[v] = 0.0;
    }
  }
};

// acc[v][a] += X[g*p + a] * y[v]; xs points at the group's values of this
// row (LDS) when p > 2, otherwise the lane's own two values are the group.
template <typename T, int P>
__device__ __forceinline__ void acc_row(LaneAcc<P>& acc, const T* xs, const T (&xo)[2], const T (&y)[2]) {
  if constexpr (P == 1) {
#pragma unroll
    for (int v = 0; v < 2; ++v) acc.a[v][0] = fma((double)xo[v], (double)y[v], acc.a[v][0]);
  } else if constexpr (P == 2) {
#pragma unroll
    for (int v = 0; v < 2; ++v)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc.a[v][j] = fma((double)xo[j], (double)y[v], acc.a[v][j]);
  } else {
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const double xv = (double)xs[j];
#pragma unroll
      for (int v = 0; v < 2; ++v) acc.a[v][j] = fma(xv, (double)y[v], acc.a[v][j]);
    }
  }
}

// out[v] = sum_a X[g*p + a] * C[a][b_v] with the lane's coefficient columns.
template <typename T, int P>
__device__ __forceinline__ void apply_row(T (&out)[2], const T* xs, const T (&xo)[2], const T (&c)[2][P]) {
  if constexpr (P == 1) {
#pragma unroll
    for (int v = 0; v < 2; ++v) out[v] = xo[v] * c[v][0];
  } else if constexpr (P == 2) {
#pragma unroll
    for (int v = 0; v < 2; ++v) out[v] = fma(xo[1], c[v][1], xo[0] * c[v][0]);
  } else {
    T s0 = T(0), s1 = T(0);
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const T xv = xs[j];
      s0 = fma(xv, c[0][j], s0);
      s1 = fma(xv, c[1][j], s1);
    }
    out[0] = s0;
    out[1] = s1;
  }
}

// Coefficient columns of this lane: c[v][a] = C_g[a][b_v] (global: C_0).
template <typename T, int P>
__device__ __forceinline__ void load_coeff(T (&c)[2][P], const T* C, int c0, int global) {
#pragma unroll
  for (int v = 0; v < 2; ++v) {
    const int col = c0 + v;
    const int g = col / P, b = col - g * P;
    const T* base = C + (global ? 0 : g * P * P) + b;
#pragma unroll
    for (int a = 0; a < P; ++a) c[v][a] = base[a * P];
  }
}

// Combines the lane partials of a workgroup and writes its packed partial row.
// H must hold K*P + K doubles of LDS.
template <int K, int P, bool NORMS>
__device__ void finish_partial(LaneAcc<P>& acc, double* H, double* prow, const Plan& pl) {
  using Gm = Geo<K, P>;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  // butterfly over the row slots of the wave (lane bits >= log2(G))
#pragma unroll
  for (int off = Gm::G; off < 64; off <<= 1) {
#pragma unroll
    for (int v = 0; v < 2; ++v) {
#pragma unroll
      for (int j = 0; j < P; ++j) acc.a[v][j] += __shfl_xor(acc.a[v][j], off);
      if (NORMS) acc.nrm[v] += __shfl_xor(acc.nrm[v], off);
    }
  }
  const int c0 = 2 * lane;  // valid for lane < G
  for (int w = 0; w < 4; ++w) {
    if (wave == w && lane < Gm::G) {
#pragma unroll
      for (int v = 0; v < 2; ++v) {
        const int col = c0 + v, g = col / P, b = col - g * P;
#pragma unroll
        for (int j = 0; j < P; ++j) {
          const int idx = g * P * P + j * P + b;
          H[idx] = (w == 0 ? 0.0 : H[idx]) + acc.a[v][j];
        }
        if (NORMS) H[K * P + col] = (w == 0 ? 0.0 : H[K * P + col]) + acc.nrm[v];
      }
    }
    __syncthreads();
  }
  const int E = pl.E;
  constexpr int PP = P * P, Q = K / P;
  for (int e = tid; e < E; e += kBlock) {
    double s;
    if (pl.global) {
      s = H[e];
      for (int g = 1; g < Q; ++g) s += H[g * PP + e];
    } else {
      s = H[e];
    }
    prow[e] = s;
  }
  if (NORMS)
    for (int j = tid; j < K; j += kBlock) prow[E + j] = H[K * P + j];
}

// ---------------------------------------------------------------- SpMM
// Indices of one row step: the CSR range and up to 8 (column, value) pairs of
// each lane's row, clamped to the row so every load is in bounds.
template <typename T>
struct RowIdx {
  int j0, j1;
  int cols[8];
  T vs[8];
};

template <typename T>
__device__ __forceinline__ void load_idx(RowIdx<T>& r, const int32_t* __restrict__ colind,
                                         const T* __restrict__ vals, int jb) {
  // entries past the row end (or of an empty row) re-read a valid entry of
  // the matrix; their products are masked out by the caller
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int jj = max(min(jb + u, r.j1 - 1), 0);
    r.cols[u] = colind[jj];
    r.vs[u] = vals[jj];
  }
}

// Broadcast of lane `src` of each aligned group of G lanes (G <= 32) through
// the LDS crossbar (ds_swizzle bit mode: lane = (lane & and) | or).
template <int G, int SRC>
__device__ __forceinline__ int bcast_i(int x) {
  static_assert(G <= 32 && SRC < G, "group broadcast within 32 lanes");
  constexpr int pattern = (SRC << 5) | (0x1F & ~(G - 1));
  return __builtin_amdgcn_ds_swizzle(x, pattern);
}

template <int G, int SRC>
__device__ __forceinline__ double bcast_v(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = bcast_i<G, SRC>(static_cast<int>(v & 0xffffffffLL));
  const int hi = bcast_i<G, SRC>(static_cast<int>(v >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

template <int G, int SRC>
__device__ __forceinline__ float bcast_v(float x) {
  return __int_as_float(bcast_i<G, SRC>(__float_as_int(x)));
}

// Cooperative index chunk: lane cg of a row group (G lanes) loads entry
// jb + cg (+ jb + cg + G for G < 8); entry u then comes from lane u % G.
template <typename T, int G>
struct CoopIdx {
  static constexpr int PER = G >= 8 ? 1 : 8 / G;
  int c[PER];
  T v[PER];
  __device__ __forceinline__ void load(const int32_t* __restrict__ colind, const T* __restrict__ vals, int jb,
                                       int j1, int cg) {
#pragma unroll
    for (int t = 0; t < PER; ++t) {
      const int jj = max(min(jb + cg + t * G, j1 - 1), 0);
      c[t] = colind[jj];
      v[t] = vals[jj];
    }
  }
  template <int U = 0>
  __device__ __forceinline__ void spread(RowIdx<T>& r) {
    if constexpr (U < 8) {
      r.cols[U] = bcast_i<G, U % G>(c[U / G]);
      r.vs[U] = bcast_v<G, U % G>(v[U / G]);
      spread<U + 1>(r);
    }
  }
};

// Q = A P with the partial alpha = <<P, Q>>. Software pipelined so that no
// wait on a younger load also waits for the current gathers (the vector
// memory counter retires loads in issue order): per step the wave issues the
// gathers of step s, then the first index chunk of step s+1 (its CSR range
// was loaded one step earlier), then the CSR range of step s+2, and only then
// consumes the gathers.
// Residual modes (FP64; Algorithm 1's initial residual, and the true residual
// of a refinement step): Pm is X, Bm is B and Q receives R = B - A X, with
// the column norms; kResidP also stores P = R (Pout) and, when the plan fuses
// products, the partial <<R, R>>.
enum FastMode { kProduct = 0, kResidual = 1, kResidP = 2 };
template <typename T, int K, int P, int MODE = kProduct>
__global__ __launch_bounds__(kBlock) void k_spmm_fast(Plan pl, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind, const T* __restrict__ vals,
                                                      const T* __restrict__ Pm, T* __restrict__ Q,
                                                      double* __restrict__ part, const DevState* st,
                                                      const T* __restrict__ Bm = nullptr,
                                                      T* __restrict__ Pout = nullptr) {
  if (halted(st)) return;
  using Gm = Geo<K, P>;
  using T2 = typename V2<T>::type;
  constexpr bool RES = MODE != kProduct;
  static_assert(!RES || sizeof(T) == 8, "the residual is formed in FP64");
  // the row slab in LDS serves the Gram of a group wider than one lane
  constexpr bool SLAB = Gm::NEED_LDS && MODE != kResidual;
  const bool gram = MODE == kProduct || (MODE == kResidP && pl.fused);
  __shared__ T slab[4][SLAB ? Gm::SLAB : 1];
  __shared__ double H[K * P + K];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int rr = lane / Gm::G, cg = lane - rr * Gm::G, c0 = 2 * cg;
  const int gcol = (c0 / P) * P;
  LaneAcc<P> acc;
  acc.zero();
  const int64_t nsteps = (pl.n + Gm::RW - 1) / Gm::RW;
  const StepRange sr = wave_steps(nsteps);
  const int64_t tw = sr.stride;
  const int64_t n = pl.n;
  // Schedule entry e = step*RW + rr names the row (natural order without a
  // schedule); entries past n (last step) use entry n-1 for their loads and
  // are discarded.
  const int32_t* __restrict__ sched = pl.sched;
  auto row_of = [&](int64_t step) -> int64_t {
    int64_t e = step * Gm::RW + rr;
    e = e < n ? e : n - 1;
    return sched ? static_cast<int64_t>(sched[e]) : e;
  };
  // all loads of the loop are unconditional (clamped rows and entries), so
  // the compiler's load-counter waits are exact; the schedule is read three
  // steps, the CSR range two steps and the index chunk one step ahead
  const int64_t last = sr.end > sr.first ? sr.end - 1 : sr.first;
  int64_t s = sr.first;
  RowIdx<T> cur;
  int64_t cur_row = 0, row1 = 0, row2 = 0;
  int nj0 = 0, nj1 = 0;  // CSR range of step s + tw
  if (s < sr.end) {
    cur_row = row_of(s);
    row1 = row_of(min(s + tw, last));
    row2 = row_of(min(s + 2 * tw, last));
    cur.j0 = rowptr[cur_row];
    cur.j1 = rowptr[cur_row + 1];
    nj0 = rowptr[row1];
    nj1 = rowptr[row1 + 1];
    if constexpr (Gm::G <= 32) {
      CoopIdx<T, Gm::G> ci;
      ci.load(colind, vals, cur.j0, cur.j1, cg);
      ci.spread(cur);
    } else {
      load_idx(cur, colind, vals, cur.j0);
    }
  }
  for (; s < sr.end; s += tw) {
    const bool ok = s * Gm::RW + rr < n;
    const int64_t i = cur_row;
    // 1. gathers of the current step and its own row of P (of B)
    T2 xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = *reinterpret_cast<const T2*>(Pm + (int64_t)cur.cols[u] * K + c0);
    const T2 pv = *reinterpret_cast<const T2*>((RES ? Bm : Pm) + i * K + c0);
    // 2. index chunk of the next step (CSR range already loaded)
    RowIdx<T> nxt;
    nxt.j0 = nj0;
    nxt.j1 = nj1;
    CoopIdx<T, (Gm::G <= 32 ? Gm::G : 32)> cnx;
    if constexpr (Gm::G <= 32)
      cnx.load(colind, vals, nj0, nj1, cg);
    else
      load_idx(nxt, colind, vals, nj0);
    // 3. CSR range two steps ahead, schedule entry three steps ahead
    nj0 = rowptr[row2];
    nj1 = rowptr[row2 + 1];
    const int64_t row3 = row_of(min(s + 3 * tw, last));
    // 4. consume the gathers
    T q[2] = {T(0), T(0)};
    {
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const bool in = cur.j0 + u < cur.j1;
        const T a0 = fma(cur.vs[u], xv[u].x, q[0]);
        const T a1 = fma(cur.vs[u], xv[u].y, q[1]);
        q[0] = in ? a0 : q[0];
        q[1] = in ? a1 : q[1];
      }
      // rows with more than 8 entries: remaining chunks without pipelining
      for (int jb = cur.j0 + 8; jb < cur.j1; jb += 8) {
        RowIdx<T> ex;
        ex.j1 = cur.j1;
        load_idx(ex, colind, vals, jb);
#pragma unroll
        for (int u = 0; u < 8; ++u) xv[u] = *reinterpret_cast<const T2*>(Pm + (int64_t)ex.cols[u] * K + c0);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const bool in = jb + u < cur.j1;
          const T a0 = fma(ex.vs[u], xv[u].x, q[0]);
          const T a1 = fma(ex.vs[u], xv[u].y, q[1]);
          q[0] = in ? a0 : q[0];
          q[1] = in ? a1 : q[1];
        }
      }
    }
    T po[2] = {T(0), T(0)};
    if constexpr (RES) {
      // R = B - A X; rows past n add nothing
      if (ok) {
        q[0] = pv.x - q[0];
        q[1] = pv.y - q[1];
        *reinterpret_cast<T2*>(Q + i * K + c0) = T2{q[0], q[1]};
        if constexpr (MODE == kResidP) *reinterpret_cast<T2*>(Pout + i * K + c0) = T2{q[0], q[1]};
      } else {
        q[0] = q[1] = T(0);
      }
      po[0] = q[0];
      po[1] = q[1];
#pragma unroll
      for (int v = 0; v < 2; ++v) acc.nrm[v] = fma(q[v], q[v], acc.nrm[v]);
    } else if (ok) {
      *reinterpret_cast<T2*>(Q + i * K + c0) = T2{q[0], q[1]};
      po[0] = pv.x;
      po[1] = pv.y;
    } else {
      q[0] = q[1] = T(0);
    }
    if constexpr (MODE != kResidual) {
      if (gram) {
        const T* xs = nullptr;
        if constexpr (SLAB) {
          T* sl = slab[wave];
          *reinterpret_cast<T2*>(sl + rr * K + c0) = T2{po[0], po[1]};
          wave_sync();
          xs = sl + rr * K + gcol;
        }
        acc_row<T, P>(acc, xs, po, q);  // alpha = <<P, Q>> (a over P, b over Q), or <<R, R>>
        if constexpr (SLAB) wave_sync();
      }
    }
    if constexpr (Gm::G <= 32) cnx.spread(nxt);
    cur = nxt;
    cur_row = row1;
    row1 = row2;
    row2 = row3;
  }
  finish_partial<K, P, RES>(acc, H, part + (int64_t)blockIdx.x * pl.W, pl);
}

// ------------------------------------------------------------ R update
// R -= Q lambda (line 9) with the partial <<R, R>> (line 11) and the column
// norms of the stop rule. X is updated later, in the pass that reads P anyway.
template <typename T, int K, int P>
__global__ __launch_bounds__(kBlock) void k_update_r_fast(Plan pl, T* __restrict__ R, const T* __restrict__ Q,
                                                          const T* __restrict__ lam, double* __restrict__ part,
                                                          const DevState* st) {
  if (fstopped(st)) return;
  using Gm = Geo<K, P>;
  using T2 = typename V2<T>::type;
  __shared__ T slab[4][2][Gm::NEED_LDS ? Gm::SLAB : 1];
  __shared__ double H[K * P + K];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int rr = lane / Gm::G, cg = lane - rr * Gm::G, c0 = 2 * cg;
  const int gcol = (c0 / P) * P;
  T cf[2][P];
  load_coeff<T, P>(cf, lam, c0, pl.global);
  LaneAcc<P> acc;
  acc.zero();
  const int64_t nsteps = (pl.n + Gm::RW - 1) / Gm::RW;
  const StepRange sr = wave_steps(nsteps);
  const int64_t tw = sr.stride;
  const int64_t n = pl.n;
  int64_t s = sr.first;
  // operands of the next row step are loaded before the current one is used
  T2 nb{}, nc{};
  if (s < sr.end) {
    const int64_t i = s * Gm::RW + rr;
    const int64_t off = (i < n ? i : n - 1) * K + c0;
    nb = *reinterpret_cast<const T2*>(Q + off);
    nc = *reinterpret_cast<const T2*>(R + off);
  }
  for (; s < sr.end; s += tw) {
    const int64_t i = s * Gm::RW + rr;
    const bool ok = i < n;
    const int64_t off = i * K + c0;
    T qv[2] = {T(0), T(0)}, rv[2] = {T(0), T(0)};
    if (ok) {
      qv[0] = nb.x; qv[1] = nb.y;
      rv[0] = nc.x; rv[1] = nc.y;
    }
    const int64_t sn = s + tw;
    if (sn < sr.end) {
      const int64_t in = sn * Gm::RW + rr;
      const int64_t offn = (in < n ? in : n - 1) * K + c0;
      nb = *reinterpret_cast<const T2*>(Q + offn);
      nc = *reinterpret_cast<const T2*>(R + offn);
    }
    const T *qs = nullptr, *rs = nullptr;
    if constexpr (Gm::NEED_LDS) {
      T* sq = slab[wave][0];
      *reinterpret_cast<T2*>(sq + rr * K + c0) = T2{qv[0], qv[1]};
      wave_sync();
      qs = sq + rr * K + gcol;
    }
    T dr[2];
    apply_row<T, P>(dr, qs, qv, cf);
    T rn[2];
#pragma unroll
    for (int v = 0; v < 2; ++v) rn[v] = rv[v] - dr[v];  // R - Q lambda
    if (ok) *reinterpret_cast<T2*>(R + off) = T2{rn[0], rn[1]};
    if constexpr (Gm::NEED_LDS) {
      T* sr2 = slab[wave][1];
      *reinterpret_cast<T2*>(sr2 + rr * K + c0) = T2{rn[0], rn[1]};
      wave_sync();
      rs = sr2 + rr * K + gcol;
    }
    acc_row<T, P>(acc, rs, rn, rn);  // <<R, R>>
#pragma unroll
    for (int v = 0; v < 2; ++v) acc.nrm[v] = fma((double)rn[v], (double)rn[v], acc.nrm[v]);
    if constexpr (Gm::NEED_LDS) wave_sync();
  }
  finish_partial<K, P, true>(acc, H, part + (int64_t)blockIdx.x * pl.W, pl);
}

// ------------------------------------------------ FP32 start of a refinement
// R32 = R64 / s with s = max_j sqrt(norms[j]) (stored to *scale), D32 = 0 and
// P32 = R32 (pfac = 0) or P32 *= pfac rounded to FP32 (residual replacement),
// with the partial <<R32, R32>> (FP64 accumulation) and the column norms.
template <int K, int P>
__global__ __launch_bounds__(kBlock) void k_cast_init_fast(Plan pl, const double* __restrict__ R64,
                                                           const double* __restrict__ norms, float* __restrict__ R32,
                                                           float* __restrict__ P32, float* __restrict__ D32,
                                                           double* __restrict__ scale, double* __restrict__ part,
                                                           double pfac) {
  using Gm = Geo<K, P>;
  __shared__ float slab[4][Gm::NEED_LDS ? Gm::SLAB : 1];
  __shared__ double H[K * P + K];
  __shared__ double s_sh;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int rr = lane / Gm::G, cg = lane - rr * Gm::G, c0 = 2 * cg;
  const int gcol = (c0 / P) * P;
  if (tid == 0) {
    double m = 0.0;
    for (int j = 0; j < K; ++j) m = fmax(m, sqrt(norms[j]));
    s_sh = m;
    if (blockIdx.x == 0) *scale = m;
  }
  __syncthreads();
  const double sc = s_sh;
  const float pf = static_cast<float>(pfac);
  LaneAcc<P> acc;
  acc.zero();
  const int64_t nsteps = (pl.n + Gm::RW - 1) / Gm::RW;
  const StepRange sr = wave_steps(nsteps);
  const int64_t n = pl.n;
  for (int64_t s = sr.first; s < sr.end; s += sr.stride) {
    const int64_t i = s * Gm::RW + rr;
    const bool ok = i < n;
    const int64_t off = (ok ? i : n - 1) * K + c0;
    const double2 r = *reinterpret_cast<const double2*>(R64 + off);
    float2 pv{0.f, 0.f};
    if (pfac != 0.0) pv = *reinterpret_cast<const float2*>(P32 + off);
    float v[2] = {0.f, 0.f};
    if (ok) {
      v[0] = static_cast<float>(r.x / sc);
      v[1] = static_cast<float>(r.y / sc);
      *reinterpret_cast<float2*>(R32 + off) = float2{v[0], v[1]};
      *reinterpret_cast<float2*>(P32 + off) = pfac == 0.0 ? float2{v[0], v[1]} : float2{pv.x * pf, pv.y * pf};
      *reinterpret_cast<float2*>(D32 + off) = float2{0.f, 0.f};
    }
    const float* vs = nullptr;
    if constexpr (Gm::NEED_LDS) {
      float* sl = slab[wave];
      *reinterpret_cast<float2*>(sl + rr * K + c0) = float2{v[0], v[1]};
      wave_sync();
      vs = sl + rr * K + gcol;
    }
    if (pl.fused) acc_row<float, P>(acc, vs, v, v);  // <<R32, R32>>
#pragma unroll
    for (int u = 0; u < 2; ++u) acc.nrm[u] = fma((double)v[u], (double)v[u], acc.nrm[u]);
    if constexpr (Gm::NEED_LDS) wave_sync();
  }
  finish_partial<K, P, true>(acc, H, part + (int64_t)blockIdx.x * pl.W, pl);
}

// ------------------------------------------------------- X and P update
// X += P lambda (line 8) and, unless this is the last iteration, P = R + P
// beta (line 13) with the partial rho = <<P_new, R>> of the next line 6. On
// the last iteration (stop rule met, iteration cap, breakdown after line 9)
// only X is updated.
template <typename T, int K, int P>
__global__ __launch_bounds__(kBlock) void k_update_xp_fast(Plan pl, T* __restrict__ X, T* __restrict__ Pm,
                                                           const T* __restrict__ R, const T* __restrict__ lam,
                                                           const T* __restrict__ beta, double* __restrict__ part,
                                                           const DevState* st) {
  if (fstopped(st)) return;
  const bool last = *reinterpret_cast<const volatile int*>(&st->last) != 0;
  using Gm = Geo<K, P>;
  using T2 = typename V2<T>::type;
  __shared__ T slab[4][2][Gm::NEED_LDS ? Gm::SLAB : 1];
  __shared__ double H[K * P + K];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int rr = lane / Gm::G, cg = lane - rr * Gm::G, c0 = 2 * cg;
  const int gcol = (c0 / P) * P;
  T cl[2][P], cb[2][P];
  load_coeff<T, P>(cl, lam, c0, pl.global);
  if (!last) load_coeff<T, P>(cb, beta, c0, pl.global);
  LaneAcc<P> acc;
  acc.zero();
  const int64_t nsteps = (pl.n + Gm::RW - 1) / Gm::RW;
  const StepRange sr = wave_steps(nsteps);
  const int64_t tw = sr.stride;
  const int64_t n = pl.n;
  int64_t s = sr.first;
  T2 na{}, nc{}, nd{};
  if (s < sr.end) {
    const int64_t i = s * Gm::RW + rr;
    const int64_t off = (i < n ? i : n - 1) * K + c0;
    na = *reinterpret_cast<const T2*>(Pm + off);
    nc = *reinterpret_cast<const T2*>(R + off);
    nd = *reinterpret_cast<const T2*>(X + off);
  }
  for (; s < sr.end; s += tw) {
    const int64_t i = s * Gm::RW + rr;
    const bool ok = i < n;
    const int64_t off = i * K + c0;
    T pv[2] = {T(0), T(0)}, rv[2] = {T(0), T(0)}, xv[2] = {T(0), T(0)};
    if (ok) {
      pv[0] = na.x; pv[1] = na.y;
      rv[0] = nc.x; rv[1] = nc.y;
      xv[0] = nd.x; xv[1] = nd.y;
    }
    const int64_t sn = s + tw;
    if (sn < sr.end) {
      const int64_t in = sn * Gm::RW + rr;
      const int64_t offn = (in < n ? in : n - 1) * K + c0;
      na = *reinterpret_cast<const T2*>(Pm + offn);
      nc = *reinterpret_cast<const T2*>(R + offn);
      nd = *reinterpret_cast<const T2*>(X + offn);
    }
    const T *ps = nullptr, *ns = nullptr;
    if constexpr (Gm::NEED_LDS) {
      T* sp = slab[wave][0];
      *reinterpret_cast<T2*>(sp + rr * K + c0) = T2{pv[0], pv[1]};
      wave_sync();
      ps = sp + rr * K + gcol;
    }
    T dx[2];
    apply_row<T, P>(dx, ps, pv, cl);
#pragma unroll
    for (int v = 0; v < 2; ++v) xv[v] = xv[v] + dx[v];  // X + P lambda
    if (ok) *reinterpret_cast<T2*>(X + off) = T2{xv[0], xv[1]};
    if (!last) {
      T dp[2];
      apply_row<T, P>(dp, ps, pv, cb);
      T pn[2];
#pragma unroll
      for (int v = 0; v < 2; ++v) pn[v] = rv[v] + dp[v];  // R + P beta
      if (ok) *reinterpret_cast<T2*>(Pm + off) = T2{pn[0], pn[1]};
      if constexpr (Gm::NEED_LDS) {
        T* sn2 = slab[wave][1];
        *reinterpret_cast<T2*>(sn2 + rr * K + c0) = T2{pn[0], pn[1]};
        wave_sync();
        ns = sn2 + rr * K + gcol;
      }
      acc_row<T, P>(acc, ns, pn, rv);  // rho = <<P_new, R>>: a over P_new, b over R
    }
    if constexpr (Gm::NEED_LDS) wave_sync();
  }
  finish_partial<K, P, false>(acc, H, part + (int64_t)blockIdx.x * pl.W, pl);
}

template <typename F>
bool dispatch_fast(const Plan& pl, F&& f) {
  auto withP = [&](auto Kc) -> bool {
    constexpr int K = decltype(Kc)::value;
    switch (pl.p) {
      case 1: f(Kc, std::integral_constant<int, 1>()); return true;
      case 2: f(Kc, std::integral_constant<int, 2>()); return true;
      case 4: if constexpr (K >= 4) { f(Kc, std::integral_constant<int, 4>()); return true; } return false;
      case 8: if constexpr (K >= 8) { f(Kc, std::integral_constant<int, 8>()); return true; } return false;
      case 16: if constexpr (K >= 16) { f(Kc, std::integral_constant<int, 16>()); return true; } return false;
      default: return false;
    }
  };
  switch (pl.k) {
    case 8: return withP(std::integral_constant<int, 8>());
    case 16: return withP(std::integral_constant<int, 16>());
    case 32: return withP(std::integral_constant<int, 32>());
    case 64: return withP(std::integral_constant<int, 64>());
    case 128: return withP(std::integral_constant<int, 128>());
    default: return false;
  }
}

}  // namespace

bool fast_supported(const Plan& pl) {
  if (std::getenv("BCG_GENERIC_ONLY") || pl.nnz < 1) return false;
  return dispatch_fast(pl, [](auto, auto) {});
}

template <typename T>
void launch_spmm_fast(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const T* vals, const T* P,
                      T* Q, double* part, const DevState* st, hipStream_t s) {
  dispatch_fast(pl, [&](auto Kc, auto Pc) {
    hipLaunchKernelGGL((k_spmm_fast<T, decltype(Kc)::value, decltype(Pc)::value>), dim3(pl.nwg), dim3(kBlock), 0, s,
                       pl, rowptr, colind, vals, P, Q, part, st);
  });
}

bool launch_residual_fast(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const double* vals,
                          const double* B, const double* X, double* R, double* P, double* part, int with_p,
                          hipStream_t s) {
  return dispatch_fast(pl, [&](auto Kc, auto Pc) {
    constexpr int K = decltype(Kc)::value, PP = decltype(Pc)::value;
    if (with_p)
      hipLaunchKernelGGL((k_spmm_fast<double, K, PP, kResidP>), dim3(pl.nwg), dim3(kBlock), 0, s, pl, rowptr, colind,
                         vals, X, R, part, nullptr, B, P);
    else
      hipLaunchKernelGGL((k_spmm_fast<double, K, PP, kResidual>), dim3(pl.nwg), dim3(kBlock), 0, s, pl, rowptr,
                         colind, vals, X, R, part, nullptr, B, nullptr);
  });
}

bool launch_cast_init_fast(const Plan& pl, const double* R64, const double* norms, float* R32, float* P32,
                           float* D32, double* scale, double* part, hipStream_t s, double pfac) {
  return dispatch_fast(pl, [&](auto Kc, auto Pc) {
    hipLaunchKernelGGL((k_cast_init_fast<decltype(Kc)::value, decltype(Pc)::value>), dim3(pl.nwg), dim3(kBlock), 0,
                       s, pl, R64, norms, R32, P32, D32, scale, part, pfac);
  });
}

template <typename T>
void launch_update_r_fast(const Plan& pl, T* R, const T* Q, const T* lam, double* part, const DevState* st,
                          hipStream_t s) {
  dispatch_fast(pl, [&](auto Kc, auto Pc) {
    hipLaunchKernelGGL((k_update_r_fast<T, decltype(Kc)::value, decltype(Pc)::value>), dim3(pl.nwg), dim3(kBlock), 0,
                       s, pl, R, Q, lam, part, st);
  });
}

template <typename T>
void launch_update_xp_fast(const Plan& pl, T* X, T* P, const T* R, const T* lam, const T* beta, double* part,
                           const DevState* st, hipStream_t s) {
  dispatch_fast(pl, [&](auto Kc, auto Pc) {
    hipLaunchKernelGGL((k_update_xp_fast<T, decltype(Kc)::value, decltype(Pc)::value>), dim3(pl.nwg), dim3(kBlock),
                       0, s, pl, X, P, R, lam, beta, part, st);
  });
}

#define BCG_FAST_INST(T)                                                                                           \
  template void launch_spmm_fast<T>(const Plan&, const int32_t*, const int32_t*, const T*, const T*, T*, double*, \
                                    const DevState*, hipStream_t);                                                 \
  template void launch_update_r_fast<T>(const Plan&, T*, const T*, const T*, double*, const DevState*,            \
                                        hipStream_t);                                                              \
  template void launch_update_xp_fast<T>(const Plan&, T*, T*, const T*, const T*, const T*, double*,              \
                                         const DevState*, hipStream_t);
BCG_FAST_INST(double)
BCG_FAST_INST(float)

}  // namespace bcg
