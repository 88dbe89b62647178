// Row kernels of the block CG iteration on the gfx950 matrix cores.
//
// For k a multiple of 16 (<= 128) every operation of an iteration on a tile
// of 16 rows is a sum of 16x16x4 FP64 matrix products (v_mfma_f64_16x16x4f64):
//   updates   Q lambda, P lambda, P beta: A = 16 rows x 4 columns of the block
//             vector, B = 4 x 16 entries of the coefficient block;
//   products  <<X, Y>>: A = 4 rows of X (as X^T), B = the same 4 rows of Y.
// Register layout of the instruction on gfx950: A (16x4) lane l holds
// A[l & 15][l >> 4]; B (4x16) lane l holds B[l >> 4][l & 15]; the result
// (16x16) lane l, element r holds D[4r + (l >> 4)][l & 15]. A result tile
// ("D layout") therefore holds, in its register r, the rows 4r..4r+3 as the
// K = 4 operand of a row reduction: block products are formed directly from
// the tiles the updates produce, with no data movement.
//
// Columns are taken in groups of width w = max(p, 16) (a whole number of
// 16-column blocks; for p < 16 a 16-column block holds 16/p groups, and the
// coefficient tiles are zero outside their p x p diagonal blocks, which adds
// exact zeros). Each wave owns one column group and walks 16-row tiles (the
// sparse product: 8-row steps); the products of its group accumulate in MFMA
// result registers and are projected onto the packed [qo][p][p] layout once
// per workgroup.
//
// FP32 block vectors (refinement inner solves) are widened to FP64 for the
// matrix products; an update is rounded to FP32 once and then applied in
// FP32, with the FP32-rounded coefficients.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <stdexcept>
#include <type_traits>

#include "../../include/bcg.h"
#include "bcg_internal.h"

namespace bcg {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Whether the row kernels may load an operand stream non-temporally: only
// where a wave's row slices cover whole 128-byte lines (see Lay).
template <typename T, int K, int PW, int GW = 1>
constexpr bool stream_nt() {
  return K == PW * GW || (PW * GW * static_cast<int>(sizeof(T))) % 128 == 0;
}

// Calls f(integral_constant<int, i>) for i = 0 .. N-1 (compile-time indices
// into per-group register arrays).
template <int N, int I = 0, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>());
    static_for<N, I + 1>(f);
  }
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
// FP32 16x16x4 product (FP32 products and accumulation). Its result lane l,
// element r holds D[4 (l >> 4) + r][l & 15] (measured on gfx950), where the
// FP64 one holds D[4r + (l >> 4)][l & 15]; the update passes feed it the A
// rows in the order tau, which gives the FP64 result layout (see load_a).
__device__ __forceinline__ f4v mfma32(float a, float b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Matrix-core products of the updates per precision: FP64 block vectors on
// the FP64 product, FP32 ones on the FP32 product (the update is an FP32
// operation on FP32 data with FP32-rounded coefficients; only the block
// products of the Grams accumulate in FP64).
template <typename T>
struct MT;
template <>
struct MT<double> {
  using acc = d4;
  __device__ static acc zero() { return d4{0.0, 0.0, 0.0, 0.0}; }
  __device__ static acc fma(double a, double b, acc c) { return mfma(a, b, c); }
};
template <>
struct MT<float> {
  using acc = f4v;
  __device__ static acc zero() { return f4v{0.0f, 0.0f, 0.0f, 0.0f}; }
  __device__ static acc fma(float a, float b, acc c) { return mfma32(a, b, c); }
};

__device__ __forceinline__ bool mstopped(const DevState* st) {
  return st != nullptr && *reinterpret_cast<const volatile int*>(&st->done) != 0;
}

template <typename T>
struct V2m;
template <>
struct V2m<double> {
  using type = double2;
};
template <>
struct V2m<float> {
  using type = float2;
};

template <int K, int PW>
struct MGeo {
  static_assert(PW % 16 == 0 && K % PW == 0, "group width");
  static constexpr int NB = PW / 16;          // 16-column blocks per group
  static constexpr int NG = K / PW;           // column groups
  static constexpr bool BREG = NB <= 2;       // coefficient operands in registers
  static constexpr int CST = PW + 4;          // LDS row stride of staged coefficients
  static constexpr int HS = NG * PW * PW;     // dense group products, then K norms
};

// Work of one wave: a fixed column group and a strided range of 16-row tiles.
// With 8 or more workgroups, each XCD (workgroup b runs on XCD b % 8) takes a
// contiguous eighth of the tiles, so neighbouring rows share its L2. Waves of
// an XCD are dealt to the groups round robin; the host guarantees at least NG
// waves per XCD (mfma_grid), and waves beyond a multiple of NG stay idle.
struct WaveWork {
  int group;
  int64_t first, end, stride;
};

template <int NG>
__device__ __forceinline__ WaveWork wave_work(int64_t ntiles) {
  const int nwg = gridDim.x, b = blockIdx.x, wave = threadIdx.x >> 6;
  int64_t lo = 0, hi = ntiles, waves, wid;
  if (nwg < 8) {
    waves = (int64_t)nwg * 4;
    wid = (int64_t)b * 4 + wave;
  } else {
    const int x = b & 7, nx = (nwg - x + 7) >> 3;
    const int64_t per = (ntiles + 7) / 8;
    lo = min((int64_t)x * per, ntiles);
    hi = min(lo + per, ntiles);
    waves = (int64_t)nx * 4;
    wid = (int64_t)(b >> 3) * 4 + wave;
  }
  const int64_t slots = waves / NG;
  WaveWork w;
  w.group = static_cast<int>(wid % NG);
  w.first = wid < slots * NG ? lo + wid / NG : hi;
  w.end = hi;
  w.stride = slots > 0 ? slots : 1;
  return w;
}

// Column order inside a 16-column block: position t holds column sigma(t) =
// 2(t&7) + (t>>3), so that lanes l and l^8 hold adjacent columns.
__device__ __forceinline__ int sigma16(int t) { return 2 * (t & 7) + (t >> 3); }
// Column order of the FP32 sparse product's operands: tau(t) = 4(t&3) + (t>>2).
__device__ __forceinline__ int tau16(int t) { return 4 * (t & 3) + (t >> 2); }
enum class Perm { sigma, tau };
// Column order of the result tiles of the updates: sigma for FP64 block
// vectors (pair layout), tau for FP32 (quad layout).
template <typename T>
__device__ __forceinline__ int ord16(int t) {
  return sizeof(T) == 8 ? sigma16(t) : tau16(t);
}
template <typename T>
constexpr Perm perm_of() {
  return sizeof(T) == 8 ? Perm::sigma : Perm::tau;
}

// Work of one wave in the chunked grid of the sparse product: workgroup b
// (XCD x = b % 8) takes a chunk of `chunk` steps per wave inside XCD x's
// contiguous eighth of the steps, so that the workgroups in flight on an XCD
// always cover a short, contiguous stretch of rows (the hardware dispatches
// them in order). With NG | 4 the waves of a workgroup share the NG column
// groups (4/NG waves each, interleaved over the chunk); otherwise each wave
// takes one group of a block of four (waves past NG stay idle).
template <int NG>
__device__ __forceinline__ WaveWork wave_work_sp(int64_t nsteps, int chunk) {
  if (chunk == 0) return wave_work<NG>(nsteps);
  constexpr bool SHARE = NG <= 4 && 4 % NG == 0;
  constexpr int NGB = SHARE ? 1 : (NG + 3) / 4, WPG = SHARE ? 4 / NG : 1;
  const int b = blockIdx.x, wave = threadIdx.x >> 6;
  const int x = b & 7, lb = b >> 3, gb = lb % NGB, c = lb / NGB;
  const int64_t per = (nsteps + 7) / 8;
  const int64_t lo = min((int64_t)x * per, nsteps), hi = min(lo + per, nsteps);
  const int64_t span = (int64_t)chunk * WPG, c0 = lo + (int64_t)c * span;
  const int G = SHARE ? wave % NG : gb * 4 + wave;
  const int widx = SHARE ? wave / NG : 0;
  const bool idle = G >= NG;
  WaveWork w;
  w.group = idle ? 0 : G;
  w.first = idle ? hi : c0 + widx;
  w.end = min(c0 + span, hi);
  w.stride = WPG;
  return w;
}

// Coefficient row of the B operand at k-step kk (pairs with load_a): FP64
// block vectors ab*16 + 8*(kk>>1) + 2*(lane>>4) + (kk&1), FP32 ab*16 +
// 4*(lane>>4) + kk (one 16-byte load per lane and block).
template <typename T>
__device__ __forceinline__ int coeff_row(int ab, int kk, int lane) {
  if constexpr (sizeof(T) == 8)
    return ab * 16 + 8 * (kk >> 1) + 2 * (lane >> 4) + (kk & 1);
  else
    return ab * 16 + 4 * (lane >> 4) + kk;
}

// B operand of coefficient block C (packed [qo][p][p]) for column group G,
// column jb*16 + sigma(lane & 15): zero outside the p x p diagonal blocks.
template <typename CT, int PW>
__device__ __forceinline__ double coeff_b(const CT* __restrict__ C, const Plan& pl, int G, int ab, int jb, int kk,
                                          int lane) {
  const int row = G * PW + coeff_row<CT>(ab, kk, lane);
  const int col = G * PW + jb * 16 + ord16<CT>(lane & 15);
  const int p = pl.p;
  const int ga = row / p, gb = col / p;
  if (ga != gb) return 0.0;
  const int g = pl.global ? 0 : ga;
  return static_cast<double>(C[(int64_t)g * p * p + (row - ga * p) * p + (col - gb * p)]);
}

// Coefficient operands of one wave: registers (w <= 32) or LDS (w = 64 = p,
// one column group per workgroup).
template <typename T, int K, int PW, int NC>
struct Coeff {
  using Gm = MGeo<K, PW>;
  static constexpr int NB = Gm::NB;
  // register copies in the coefficients' own precision (FP32 coefficients
  // are FP32-rounded values, widened exactly at each use)
  T r[NC][Gm::BREG ? NB * NB * 4 : 1];
  const double* lds;

  // Called by every thread of the workgroup.
  __device__ __forceinline__ void load(const T* const (&C)[NC], const bool (&use)[NC], const Plan& pl, int G,
                                       double* smem) {
    const int lane = threadIdx.x & 63;
    if constexpr (Gm::BREG) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int ab = 0; ab < NB; ++ab)
#pragma unroll
          for (int jb = 0; jb < NB; ++jb)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk)
              r[c][(ab * NB + jb) * 4 + kk] = use[c] ? static_cast<T>(coeff_b<T, PW>(C[c], pl, G, ab, jb, kk, lane)) : T(0);
    } else {
      static_assert(Gm::NG == 1, "LDS-staged coefficients need one group per workgroup");
      for (int c = 0; c < NC; ++c) {
        const T* src = C[c] + (pl.global ? 0 : (int64_t)G * PW * PW);
        for (int e = threadIdx.x; e < PW * PW; e += kBlock) {
          const int a = e / PW, b = e - a * PW;
          smem[c * PW * Gm::CST + a * Gm::CST + b] = use[c] ? static_cast<double>(src[e]) : 0.0;
        }
      }
      lds = smem;
      __syncthreads();
    }
  }
  __device__ __forceinline__ double b(int c, int ab, int jb, int kk, int lane) const {
    if constexpr (Gm::BREG) {
      return static_cast<double>(r[c][(ab * NB + jb) * 4 + kk]);
    } else {
      return lds[c * PW * Gm::CST + coeff_row<T>(ab, kk, lane) * Gm::CST + jb * 16 + ord16<T>(lane & 15)];
    }
  }
  // the operand in the block vectors' precision (FP32: the FP32-rounded value)
  __device__ __forceinline__ T bt(int c, int ab, int jb, int kk, int lane) const {
    if constexpr (Gm::BREG)
      return r[c][(ab * NB + jb) * 4 + kk];
    else
      return static_cast<T>(b(c, ab, jb, kk, lane));
  }
};

// Value of lane l^8 (DPP row_ror:8 within each row of 16 lanes).
__device__ __forceinline__ int xch(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);
}
__device__ __forceinline__ float xch(float x) { return __int_as_float(xch(__float_as_int(x))); }
__device__ __forceinline__ double xch(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = xch(static_cast<int>(v & 0xffffffffLL));
  const int hi = xch(static_cast<int>(v >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// A operand of block ab: lane l holds row (l & 15) of the tile at the
// columns coeff_row gives for k-steps kk = 0..3 (FP64: two 16-byte loads,
// FP32: one). Rows past n read row n-1 and are zeroed. Non-temporal where
// stream_nt allows: the operand (Q in the R update, the old P in the X/P
// pass) is dead after it.
//
// FP64: each of the two loads covers whole 128-byte lines (8 rows x 16
// doubles). Load h reads rows 8h .. 8h + 7: a lane whose bit 3 equals h reads
// its own row's first pair (columns 2s, 2s + 1, s = l >> 4); the other lanes
// read the second pair (columns 8 + 2s, 8 + 2s + 1) of the row of lane l ^ 8,
// which one DPP swap between lanes l and l ^ 8 delivers. (Loading each
// lane's own row twice covers only half of each line per instruction; with
// non-temporal loads every half-line then costs its own DRAM access.)
//
// FP32 (the operand of the FP32 product): lane l holds tile row tau(l & 15),
// so that the product's result tile comes out in the FP64 layout.
template <typename T, int K, int PW, bool NT>
__device__ __forceinline__ void load_a(T (&a)[4], const T* __restrict__ X, int64_t row0, int64_t n, int G, int ab,
                                       int lane) {
  const int64_t r = row0 + (sizeof(T) == 8 ? (lane & 15) : tau16(lane & 15));
  const bool ok = r < n;
  if constexpr (sizeof(T) == 8) {
    const int s = lane >> 4, b3 = (lane >> 3) & 1;
    d2v u[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t rh = min(row0 + (lane & 7) + 8 * h, n - 1);
      const T* src = X + rh * K + G * PW + ab * 16 + (b3 == h ? 2 * s : 8 + 2 * s);
      if constexpr (NT)
        u[h] = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(src));
      else
        u[h] = *reinterpret_cast<const d2v*>(src);
    }
    const d2v own = b3 ? u[1] : u[0], w = b3 ? u[0] : u[1];
    const double o0 = xch(w.x), o1 = xch(w.y);
    a[0] = ok ? own.x : 0.0;
    a[1] = ok ? own.y : 0.0;
    a[2] = ok ? o0 : 0.0;
    a[3] = ok ? o1 : 0.0;
  } else {
    const int64_t rc = ok ? r : n - 1;
    const f4v* src = reinterpret_cast<const f4v*>(X + rc * K + G * PW + ab * 16 + 4 * (lane >> 4));
    f4v v;
    if constexpr (NT)
      v = __builtin_nontemporal_load(src);
    else
      v = *src;
    a[0] = ok ? v.x : 0.0f;
    a[1] = ok ? v.y : 0.0f;
    a[2] = ok ? v.z : 0.0f;
    a[3] = ok ? v.w : 0.0f;
  }
}

// Whole-line accesses of two adjacent 16-column FP32 groups (columns c0 ..
// c0 + 31, one 128-byte line of each row) of a 16-row tile. Each of the two
// instructions of an access covers 8 rows of both groups: 8 whole lines.
// A lane's values of both groups stay in the layouts the products use; the
// lane whose bit 3 differs from the instruction's index h moves the second
// group's values of the row of lane l ^ 8 instead of its own, and one DPP
// swap between lanes l and l ^ 8 delivers them. Addresses are the tile's
// first row Mt (uniform) plus a 32-bit lane offset; rows past lim (the last
// row below n, relative to the tile) read row lim and are not stored.
template <bool NT>
__device__ __forceinline__ f4v pair_ld(const float* Mt, int off) {
  const f4v* src = reinterpret_cast<const f4v*>(reinterpret_cast<const char*>(Mt) + static_cast<uint32_t>(off) * 4u);
  if constexpr (NT)
    return __builtin_nontemporal_load(src);
  else
    return *src;
}
template <bool NT>
__device__ __forceinline__ void pair_st(float* Mt, int off, f4v v) {
  f4v* dst = reinterpret_cast<f4v*>(reinterpret_cast<char*>(Mt) + static_cast<uint32_t>(off) * 4u);
  if constexpr (NT)
    __builtin_nontemporal_store(v, dst);
  else
    *dst = v;
}

// A operands of the FP32 product: lane l holds tile row tau(l & 15) =
// 4 (l & 3) + ((l >> 2) & 3) (the order under which the product's result tile
// has the FP64 layout), columns 4s .. 4s + 3 (s = l >> 4) of each group; rows
// past lim are zeroed. A lane's row lies in half h = bit 1 of l, so here the
// lane whose bit 1 differs from the instruction's index moves the
// second group's quad of the row of lane l ^ 2, and a DPP quad permutation
// delivers it.
__device__ __forceinline__ float qswap(float x) {  // value of lane l ^ 2
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));
}
template <bool NT>
__device__ __forceinline__ void pair_load_a(float (&a0)[4], float (&a1)[4], const float* Mt, int lim, int K, int c0,
                                            int lane) {
  const int b1 = (lane >> 1) & 1;
  const int row = tau16(lane & 15), prow = tau16((lane ^ 2) & 15);
  f4v u[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
    u[h] = pair_ld<NT>(Mt, min(b1 == h ? row : prow, lim) * K + c0 + (b1 == h ? 0 : 16) + 4 * (lane >> 4));
  const f4v own = b1 ? u[1] : u[0], w = b1 ? u[0] : u[1];
  const bool ok = row <= lim;
  const float o[4] = {qswap(w.x), qswap(w.y), qswap(w.z), qswap(w.w)};
  const float m[4] = {own.x, own.y, own.z, own.w};
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    a0[e] = ok ? m[e] : 0.0f;
    a1[e] = ok ? o[e] : 0.0f;
  }
}

// Row-layout values (the FP32 quad layout of the updates: lane l holds row
// 4t + s, t = (l >> 2) & 3, s = l >> 4, columns 4c .. 4c + 3, c = l & 3, of
// each group). Instruction h moves rows 8h .. 8h + 7 (t = 2h, 2h + 1).
__device__ __forceinline__ int pair_row(int h, int lane) { return 4 * (2 * h + ((lane >> 2) & 1)) + (lane >> 4); }
template <bool NT>
__device__ __forceinline__ void pair_load(float (&g0)[4], float (&g1)[4], const float* Mt, int lim, int K, int c0,
                                          int lane) {
  const int b3 = (lane >> 3) & 1;
  f4v u[2];
#pragma unroll
  for (int h = 0; h < 2; ++h)
    u[h] = pair_ld<NT>(Mt, min(pair_row(h, lane), lim) * K + c0 + (b3 == h ? 0 : 16) + 4 * (lane & 3));
  const f4v own = b3 ? u[1] : u[0], w = b3 ? u[0] : u[1];
  g0[0] = own.x;
  g0[1] = own.y;
  g0[2] = own.z;
  g0[3] = own.w;
  g1[0] = xch(w.x);
  g1[1] = xch(w.y);
  g1[2] = xch(w.z);
  g1[3] = xch(w.w);
}
// Stores the rows up to lim (values in the quad layout of both groups).
template <bool NT>
__device__ __forceinline__ void pair_store(float* Mt, const float (&g0)[4], const float (&g1)[4], int lim, int K,
                                           int c0, int lane) {
  const int b3 = (lane >> 3) & 1;
  const f4v own = {g0[0], g0[1], g0[2], g0[3]};
  const f4v w = {xch(g1[0]), xch(g1[1]), xch(g1[2]), xch(g1[3])};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = pair_row(h, lane);
    if (r <= lim) pair_st<NT>(Mt, r * K + c0 + (b3 == h ? 0 : 16) + 4 * (lane & 3), b3 == h ? own : w);
  }
}

// Last row below n of the tile starting at row0, relative to it (0..15).
__device__ __forceinline__ int tile_lim(int64_t row0, int64_t n) {
  const int64_t l = n - 1 - row0;
  return l < 15 ? static_cast<int>(l) : 15;
}

// 4 x 4 transpose among lanes l, l^4, l^8, l^12 (t = (l>>2)&3): in v[e] =
// M[t][e], out w[m] = M[m][t] (three XOR swizzles within each 32 lanes).
template <int D>
__device__ __forceinline__ float xor4(float x) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(x), ((4 * D) << 10) | 0x1F));
}
// a_i selected by the two bits of i, on values: two levels of selects. (A
// compare chain compiles to branches, and selects between elements of one
// array can be folded into an indexed access that moves the array to LDS.)
__device__ __forceinline__ float sel4(float a0, float a1, float a2, float a3, int i) {
  const float lo = (i & 1) ? a1 : a0, hi = (i & 1) ? a3 : a2;
  return (i & 2) ? hi : lo;
}
__device__ __forceinline__ void transpose4(const float (&v)[4], float (&w)[4], int t) {
  const float v0 = v[0], v1 = v[1], v2 = v[2], v3 = v[3];
  const float s1 = xor4<1>(sel4(v0, v1, v2, v3, t ^ 1)), s2 = xor4<2>(sel4(v0, v1, v2, v3, t ^ 2)),
              s3 = xor4<3>(sel4(v0, v1, v2, v3, t ^ 3));
  const float own = sel4(v0, v1, v2, v3, t);
  w[0] = sel4(own, s1, s2, s3, t);
  w[1] = sel4(own, s1, s2, s3, t ^ 1);
  w[2] = sel4(own, s1, s2, s3, t ^ 2);
  w[3] = sel4(own, s1, s2, s3, t ^ 3);
}

// Row layouts of a 16 x 16 tile for 2- or 4-element row accesses. A result
// tile (element r: row 4r + s, s = l>>4, column ord16(l&15)) is converted by
// to_rows and back, for the block products, by from_rows.
//   FP64, pair layout: lane l (c = l&7, odd = bit 3) holds columns 2c, 2c+1
//     of rows 4(2 odd + m) + s, m = 0, 1; one exchange of two values between
//     lanes l and l^8 (sigma order: lanes l, l^8 hold adjacent columns).
//   FP32, quad layout: lane l (c = l&3, t = (l>>2)&3) holds columns 4c..4c+3
//     of row 4t + s; a 4 x 4 transpose among lanes l, l^4, l^8, l^12 (tau
//     order: these lanes hold columns 4c..4c+3).
// v[m * NC + e] is row slot m, column e.
template <typename T>
struct Lay;
// Cache policy of the row kernels' streams: an operand that no later kernel of
// the iteration reads is loaded (and X stored) non-temporally, which leaves
// the L2 and the 256 MB memory-side cache to what the next kernel reads: R
// written by the R update, P written by the X/P pass, Q, and A. This is Q and R
// in the R update, and X, the old P and R in the X/P pass (headline solve
// 117.0 -> 108.2 ms). Two conditions:
// - a wave's row slices cover whole 128-byte lines (the group spans the row,
//   or its slice is a multiple of 128 bytes; stream_nt): a line shared with
//   another wave's columns would be evicted before that wave reads its half
//   (FP32, k = 64, 16-column groups: X/P pass 624 -> 915 us);
// - the iteration's operands exceed the memory-side cache (Plan::nt): when
//   they fit, everything stays cached anyway (FP32, 512^2, k = 32: 179 ->
//   187 ms with non-temporal streams).
template <>
struct Lay<double> {
  template <bool NT>
  __device__ static void load_p(const double* p, double* v) {
    if constexpr (NT)
      load_nt(p, v);
    else
      load(p, v);
  }
  template <bool NT>
  __device__ static void store_p(double* p, const double* v) {
    if constexpr (NT)
      store_nt(p, v);
    else
      store(p, v);
  }
  __device__ static void load_nt(const double* p, double* v) {
    const d2v x = __builtin_nontemporal_load(reinterpret_cast<const d2v*>(p));
    v[0] = x.x;
    v[1] = x.y;
  }
  __device__ static void store_nt(double* p, const double* v) {
    const d2v x = {v[0], v[1]};
    __builtin_nontemporal_store(x, reinterpret_cast<d2v*>(p));
  }
  static constexpr int NR = 2, NC = 2;
  __device__ static int row(int m, int lane) { return 4 * (2 * ((lane >> 3) & 1) + m) + (lane >> 4); }
  __device__ static int col(int lane) { return 2 * (lane & 7); }
  __device__ static void load(const double* p, double* v) {
    const double2 x = *reinterpret_cast<const double2*>(p);
    v[0] = x.x;
    v[1] = x.y;
  }
  __device__ static void store(double* p, const double* v) { *reinterpret_cast<double2*>(p) = double2{v[0], v[1]}; }
};
template <>
struct Lay<float> {
  template <bool NT>
  __device__ static void load_p(const float* p, float* v) {
    if constexpr (NT)
      load_nt(p, v);
    else
      load(p, v);
  }
  template <bool NT>
  __device__ static void store_p(float* p, const float* v) {
    if constexpr (NT)
      store_nt(p, v);
    else
      store(p, v);
  }
  __device__ static void load_nt(const float* p, float* v) {
    const f4v x = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
    v[0] = x.x;
    v[1] = x.y;
    v[2] = x.z;
    v[3] = x.w;
  }
  __device__ static void store_nt(float* p, const float* v) {
    const f4v x = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(x, reinterpret_cast<f4v*>(p));
  }
  static constexpr int NR = 1, NC = 4;
  __device__ static int row(int, int lane) { return 4 * ((lane >> 2) & 3) + (lane >> 4); }
  __device__ static int col(int lane) { return 4 * (lane & 3); }
  __device__ static void load(const float* p, float* v) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    v[0] = x.x;
    v[1] = x.y;
    v[2] = x.z;
    v[3] = x.w;
  }
  __device__ static void store(float* p, const float* v) {
    *reinterpret_cast<float4*>(p) = float4{v[0], v[1], v[2], v[3]};
  }
};

__device__ __forceinline__ void to_rows(const d4& D, double (&v)[4], int lane) {
  const bool odd = (lane >> 3) & 1;
  const double r0 = xch(odd ? D[0] : D[2]), r1 = xch(odd ? D[1] : D[3]);
  v[0] = odd ? r0 : D[0];
  v[1] = odd ? D[2] : r0;
  v[2] = odd ? r1 : D[1];
  v[3] = odd ? D[3] : r1;
}
__device__ __forceinline__ void from_rows(const double (&v)[4], double (&x)[4], int lane) {
  const bool odd = (lane >> 3) & 1;
  const double r0 = xch(odd ? v[0] : v[1]), r1 = xch(odd ? v[2] : v[3]);
  x[0] = odd ? r0 : v[0];
  x[1] = odd ? r1 : v[2];
  x[2] = odd ? v[1] : r0;
  x[3] = odd ? v[3] : r1;
}
__device__ __forceinline__ void to_rows(const d4& D, float (&v)[4], int lane) {
  const float d[4] = {static_cast<float>(D[0]), static_cast<float>(D[1]), static_cast<float>(D[2]),
                      static_cast<float>(D[3])};
  transpose4(d, v, (lane >> 2) & 3);
}
__device__ __forceinline__ void to_rows(const f4v& D, float (&v)[4], int lane) {
  const float d[4] = {D[0], D[1], D[2], D[3]};
  transpose4(d, v, (lane >> 2) & 3);
}
__device__ __forceinline__ void from_rows(const float (&v)[4], double (&x)[4], int lane) {
  float w[4];
  transpose4(v, w, (lane >> 2) & 3);
#pragma unroll
  for (int r = 0; r < 4; ++r) x[r] = static_cast<double>(w[r]);
}

// Per-wave partial block products: result tiles per block pair.
template <int NB>
struct MAcc {
  d4 g[NB * NB];
  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < NB * NB; ++i) g[i] = d4{0.0, 0.0, 0.0, 0.0};
  }
};

// acc(ab, jb) += X_tile[ab]^T Y_tile[jb] over 16 rows, operands in the
// sigma-ordered result layout (register r: rows 4r + (l>>4)).
template <int NB>
__device__ __forceinline__ void gram_tiles(MAcc<NB>& acc, const double (&x)[NB][4], const double (&y)[NB][4]) {
#pragma unroll
  for (int ab = 0; ab < NB; ++ab)
#pragma unroll
    for (int jb = 0; jb < NB; ++jb)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc.g[ab * NB + jb] = mfma(x[ab][r], y[jb][r], acc.g[ab * NB + jb]);
}

// Combines the wave partials of the workgroup in a fixed order and writes the
// packed partial row [qo][p][p] (NORMS: + the k column norms, the diagonal of
// the product <<R, R>>). The tiles hold rows and columns in sigma order within
// each 16-column block (tau order for the FP32 sparse product). H: HS + K
// doubles of LDS.
template <int K, int PW, bool NORMS, Perm PM = Perm::sigma, int GW = 1>
__device__ void finish_mfma(MAcc<PW / 16> (&acc)[GW], int G0, double* H, double* prow, const Plan& pl) {
  using Gm = MGeo<K, PW>;
  constexpr int NB = Gm::NB, HS = Gm::HS;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  __syncthreads();  // staged coefficients may share this memory
  for (int e = tid; e < HS + K; e += kBlock) H[e] = 0.0;
  __syncthreads();
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int g = 0; g < GW; ++g) {
        double* HG = H + (G0 + g) * PW * PW;
#pragma unroll
        for (int ab = 0; ab < NB; ++ab)
#pragma unroll
          for (int jb = 0; jb < NB; ++jb)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int ti = PM == Perm::sigma ? sigma16(4 * r + (lane >> 4)) : tau16(4 * r + (lane >> 4));
              const int tj = PM == Perm::sigma ? sigma16(lane & 15) : tau16(lane & 15);
              HG[(ab * 16 + ti) * PW + jb * 16 + tj] += acc[g].g[ab * NB + jb][r];
            }
      }
    }
    __syncthreads();
  }
  const int p = pl.p, pp = p * p;
  for (int e = tid; e < pl.E; e += kBlock) {
    const int g0 = e / pp, rem = e - g0 * pp, a = rem / p, b = rem - a * p;
    const int gfirst = pl.global ? 0 : g0, glast = pl.global ? pl.q : g0 + 1;
    double s = 0.0;
    for (int g = gfirst; g < glast; ++g) {
      const int ca = g * p + a, cb = g * p + b, Gi = ca / PW;
      s += H[Gi * PW * PW + (ca - Gi * PW) * PW + (cb - Gi * PW)];
    }
    prow[e] = s;
  }
  if (NORMS)
    for (int c = tid; c < K; c += kBlock) {
      const int Gi = c / PW, cl = c - Gi * PW;
      prow[pl.E + c] = H[Gi * PW * PW + cl * PW + cl];
    }
}

template <int K, int PW, bool NORMS, Perm PM = Perm::sigma>
__device__ __forceinline__ void finish_mfma(MAcc<PW / 16>& acc, int G, double* H, double* prow, const Plan& pl) {
  MAcc<PW / 16> one[1] = {acc};
  finish_mfma<K, PW, NORMS, PM, 1>(one, G, H, prow, pl);
}

template <int K, int PW, int NC>
constexpr int smem_doubles() {
  using Gm = MGeo<K, PW>;
  constexpr int h = Gm::HS + K, c = Gm::BREG ? 0 : NC * PW * Gm::CST;
  return h > c ? h : c;
}

// ------------------------------------------------------------ R update
// R -= Q lambda (line 9) and the partial <<R, R>> (line 11), whose diagonal
// gives the column norms of the stop rule. A wave takes GW adjacent column
// groups of each of its tiles, one after the other: with GW PW-column groups
// covering a whole 128-byte line of every row, no line is shared with
// another wave and the streams may be non-temporal (FP32, 16-column groups:
// GW = 2). FP32 with single-block groups: the operands of the next unit (a
// tile's next group, or the next tile's first) are loaded before the products
// of the current one (on the last tile of a wave the current tile is loaded
// again, from cache); FP64 moves twice the bytes per product and gains
// nothing from it.
template <typename T, int K, int PW, bool NT, int GW>
__global__ __launch_bounds__(kBlock) void k_update_r_mfma(Plan pl, T* __restrict__ R, const T* __restrict__ Q,
                                                          const T* __restrict__ lam, double* __restrict__ part,
                                                          const DevState* st) {
  if (mstopped(st)) return;
  using Gm = MGeo<K, PW>;
  using L = Lay<T>;
  constexpr int NB = Gm::NB;
  static_assert(Gm::NG % GW == 0 && (GW == 1 || Gm::BREG), "groups per wave");
  __shared__ double smem[smem_doubles<K, PW, 1>()];
  const int lane = threadIdx.x & 63;
  const int64_t n = pl.n;
  const WaveWork ww = wave_work<Gm::NG / GW>((n + 15) / 16);
  const int G0 = ww.group * GW;
  Coeff<T, K, PW, 1> cf[GW];
#pragma unroll
  for (int g = 0; g < GW; ++g) cf[g].load({lam}, {true}, pl, G0 + g, smem);
  MAcc<NB> acc[GW];
#pragma unroll
  for (int g = 0; g < GW; ++g) acc[g].zero();
  T qa[NB][4];
  T ra[NB][4];
  auto load_rows = [&](int64_t t, int G, int jb, T (&r)[4]) {
    const int cbase = G * PW + L::col(lane);
#pragma unroll
    for (int m = 0; m < L::NR; ++m) {
      const int64_t row = min(t * 16 + L::row(m, lane), n - 1);
      L::template load_p<NT>(R + row * K + cbase + jb * 16, r + m * L::NC);
    }
  };
  auto load_unit = [&](int64_t t, int G, T (&q)[NB][4], T (&r)[NB][4]) {
#pragma unroll
    for (int ab = 0; ab < NB; ++ab) load_a<T, K, PW, NT>(q[ab], Q, t * 16, n, G, ab, lane);
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) load_rows(t, G, jb, r[jb]);
  };
  constexpr bool PIPE = sizeof(T) == 4 && NB == 1;
  if constexpr (sizeof(T) == 4 && GW == 2 && NB == 1) {
    // both groups of a tile at once, every access a whole line of each row
    const int c0 = G0 * PW;
    float q2[2][4], r2[2][4];
    auto load_pair = [&](int64_t t, float (&q)[2][4], float (&r)[2][4]) {
      const int lim = tile_lim(t * 16, n);
      pair_load_a<NT>(q[0], q[1], Q + t * 16 * K, lim, K, c0, lane);
      pair_load<NT>(r[0], r[1], R + t * 16 * K, lim, K, c0, lane);
    };
    if (ww.first < ww.end) load_pair(ww.first, q2, r2);
    for (int64_t t = ww.first; t < ww.end; t += ww.stride) {
      const int64_t row0 = t * 16;
      float qn[2][4], rnx[2][4];
      load_pair(t + ww.stride < ww.end ? t + ww.stride : t, qn, rnx);
      const bool ok = row0 + L::row(0, lane) < n;
      float rv[2][4];
      double rn[2][1][4];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        f4v D = MT<float>::zero();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) D = mfma32(q2[g][kk], cf[g].bt(0, 0, 0, kk, lane), D);
        float dq[4];
        to_rows(D, dq, lane);
#pragma unroll
        for (int e = 0; e < 4; ++e) rv[g][e] = ok ? r2[g][e] - dq[e] : 0.0f;  // R - Q lambda
        from_rows(rv[g], rn[g][0], lane);
      }
      pair_store<false>(R + row0 * K, rv[0], rv[1], tile_lim(row0, n), K, c0, lane);
#pragma unroll
      for (int g = 0; g < 2; ++g) gram_tiles<1>(acc[g], rn[g], rn[g]);
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          q2[g][e] = qn[g][e];
          r2[g][e] = rnx[g][e];
        }
    }
  } else {
  if (PIPE && ww.first < ww.end) load_unit(ww.first, G0, qa, ra);
  for (int64_t t = ww.first; t < ww.end; t += ww.stride) {
    const int64_t row0 = t * 16;
    static_for<GW>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      const int G = G0 + g;
      const int cbase = G * PW + L::col(lane);
      T qn[NB][4];
      T rnx[NB][4];
      if constexpr (PIPE) {
        if constexpr (g + 1 < GW)
          load_unit(t, G + 1, qn, rnx);
        else
          load_unit(t + ww.stride < ww.end ? t + ww.stride : t, G0, qn, rnx);
      } else {
#pragma unroll
        for (int ab = 0; ab < NB; ++ab) load_a<T, K, PW, NT>(qa[ab], Q, row0, n, G, ab, lane);
      }
      double rn[NB][4];
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        auto D = MT<T>::zero();
#pragma unroll
        for (int ab = 0; ab < NB; ++ab)
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) D = MT<T>::fma(qa[ab][kk], cf[g].bt(0, ab, jb, kk, lane), D);
        if constexpr (!PIPE) load_rows(t, G, jb, ra[jb]);
        T dq[4], rv[4];
        to_rows(D, dq, lane);
#pragma unroll
        for (int m = 0; m < L::NR; ++m) {
          const int64_t row = row0 + L::row(m, lane);
          const bool ok = row < n;
          T* v = rv + m * L::NC;
#pragma unroll
          for (int e = 0; e < L::NC; ++e) v[e] = ok ? ra[jb][m * L::NC + e] - dq[m * L::NC + e] : T(0);  // R - Q lambda
          if (ok) L::store(R + row * K + cbase + jb * 16, v);
        }
        from_rows(rv, rn[jb], lane);
      }
      gram_tiles<NB>(acc[g], rn, rn);
      if constexpr (PIPE)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            qa[jb][e] = qn[jb][e];
            ra[jb][e] = rnx[jb][e];
          }
    });
  }
  }
  finish_mfma<K, PW, true, perm_of<T>(), GW>(acc, G0, smem, part + (int64_t)blockIdx.x * pl.W, pl);
}

// ------------------------------------------------------- X and P update
// X += P lambda (line 8); unless `last`: P = R + P beta (line 13) and the
// partial rho = <<P_new, R>> of the next iteration's line 6. Groups per wave
// and pipelining as in the R update.
template <typename T, int K, int PW, bool NT, int GW>
__global__ __launch_bounds__(kBlock) void k_update_xp_mfma(Plan pl, T* __restrict__ X, T* __restrict__ Pm,
                                                           const T* __restrict__ R, const T* __restrict__ lam,
                                                           const T* __restrict__ beta, double* __restrict__ part,
                                                           const DevState* st) {
  if (mstopped(st)) return;
  const bool last = *reinterpret_cast<const volatile int*>(&st->last) != 0;
  using Gm = MGeo<K, PW>;
  using L = Lay<T>;
  constexpr int NB = Gm::NB;
  static_assert(Gm::NG % GW == 0 && (GW == 1 || Gm::BREG), "groups per wave");
  __shared__ double smem[smem_doubles<K, PW, 2>()];
  const int lane = threadIdx.x & 63;
  const int64_t n = pl.n;
  const WaveWork ww = wave_work<Gm::NG / GW>((n + 15) / 16);
  const int G0 = ww.group * GW;
  Coeff<T, K, PW, 2> cf[GW];
#pragma unroll
  for (int g = 0; g < GW; ++g) cf[g].load({lam, beta}, {true, !last}, pl, G0 + g, smem);
  MAcc<NB> acc[GW];
#pragma unroll
  for (int g = 0; g < GW; ++g) acc[g].zero();
  T pa[NB][4];
  T xa[NB][4], ra[NB][4];
  auto load_rows = [&](int64_t t, int G, int jb, T (&x)[4], T (&r)[4]) {
    const int cbase = G * PW + L::col(lane);
#pragma unroll
    for (int m = 0; m < L::NR; ++m) {
      const int64_t off = min(t * 16 + L::row(m, lane), n - 1) * K + cbase + jb * 16;
      L::template load_p<NT>(X + off, x + m * L::NC);
      if (!last) L::template load_p<NT>(R + off, r + m * L::NC);
    }
  };
  auto load_unit = [&](int64_t t, int G, T (&pq)[NB][4], T (&x)[NB][4], T (&r)[NB][4]) {
#pragma unroll
    for (int ab = 0; ab < NB; ++ab) load_a<T, K, PW, NT>(pq[ab], Pm, t * 16, n, G, ab, lane);
#pragma unroll
    for (int jb = 0; jb < NB; ++jb) load_rows(t, G, jb, x[jb], r[jb]);
  };
  constexpr bool PIPE = sizeof(T) == 4 && NB == 1;
  if constexpr (sizeof(T) == 4 && GW == 2 && NB == 1) {
    // both groups of a tile at once, every access a whole line of each row
    const int c0 = G0 * PW;
    float p2[2][4], x2[2][4], r2[2][4];
    auto load_pair = [&](int64_t t, float (&pq)[2][4], float (&x)[2][4], float (&r)[2][4]) {
      const int lim = tile_lim(t * 16, n);
      pair_load_a<NT>(pq[0], pq[1], Pm + t * 16 * K, lim, K, c0, lane);
      pair_load<NT>(x[0], x[1], X + t * 16 * K, lim, K, c0, lane);
      if (!last) pair_load<NT>(r[0], r[1], R + t * 16 * K, lim, K, c0, lane);
    };
    if (ww.first < ww.end) load_pair(ww.first, p2, x2, r2);
    for (int64_t t = ww.first; t < ww.end; t += ww.stride) {
      const int64_t row0 = t * 16;
      float pnx[2][4], xnx[2][4], rnx[2][4];
      load_pair(t + ww.stride < ww.end ? t + ww.stride : t, pnx, xnx, rnx);
      const bool ok = row0 + L::row(0, lane) < n;
      float xv[2][4], pv[2][4], rv[2][4];
      double pn[2][1][4], rd[2][1][4];
#pragma unroll
      for (int g = 0; g < 2; ++g) {
        f4v Dx = MT<float>::zero(), Dp = MT<float>::zero();
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) Dx = mfma32(p2[g][kk], cf[g].bt(0, 0, 0, kk, lane), Dx);
        float dx[4], dp[4] = {0.0f, 0.0f, 0.0f, 0.0f};
        to_rows(Dx, dx, lane);
        if (!last) {
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) Dp = mfma32(p2[g][kk], cf[g].bt(1, 0, 0, kk, lane), Dp);
          to_rows(Dp, dp, lane);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          xv[g][e] = x2[g][e] + dx[e];  // X + P lambda
          rv[g][e] = (ok && !last) ? r2[g][e] : 0.0f;
          pv[g][e] = (ok && !last) ? rv[g][e] + dp[e] : 0.0f;  // R + P beta
        }
      }
      const int lim = tile_lim(row0, n);
      pair_store<NT>(X + row0 * K, xv[0], xv[1], lim, K, c0, lane);
      if (!last) {
        pair_store<false>(Pm + row0 * K, pv[0], pv[1], lim, K, c0, lane);
#pragma unroll
        for (int g = 0; g < 2; ++g) {
          from_rows(pv[g], pn[g][0], lane);
          from_rows(rv[g], rd[g][0], lane);
          gram_tiles<1>(acc[g], pn[g], rd[g]);  // rho = <<P_new, R>>
        }
      }
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          p2[g][e] = pnx[g][e];
          x2[g][e] = xnx[g][e];
          r2[g][e] = rnx[g][e];
        }
    }
  } else {
  if (PIPE && ww.first < ww.end) load_unit(ww.first, G0, pa, xa, ra);
  for (int64_t t = ww.first; t < ww.end; t += ww.stride) {
    const int64_t row0 = t * 16;
    static_for<GW>([&](auto gc) {
      constexpr int g = decltype(gc)::value;
      const int G = G0 + g;
      const int cbase = G * PW + L::col(lane);
      T pnx[NB][4];
      T xnx[NB][4], rnx[NB][4];
      if constexpr (PIPE) {
        if constexpr (g + 1 < GW)
          load_unit(t, G + 1, pnx, xnx, rnx);
        else
          load_unit(t + ww.stride < ww.end ? t + ww.stride : t, G0, pnx, xnx, rnx);
      } else {
#pragma unroll
        for (int ab = 0; ab < NB; ++ab) load_a<T, K, PW, NT>(pa[ab], Pm, row0, n, G, ab, lane);
      }
      double pn[NB][4], rd[NB][4];
#pragma unroll
      for (int jb = 0; jb < NB; ++jb) {
        auto Dx = MT<T>::zero(), Dp = MT<T>::zero();
#pragma unroll
        for (int ab = 0; ab < NB; ++ab)
#pragma unroll
          for (int kk = 0; kk < 4; ++kk) Dx = MT<T>::fma(pa[ab][kk], cf[g].bt(0, ab, jb, kk, lane), Dx);
        if constexpr (!PIPE) load_rows(t, G, jb, xa[jb], ra[jb]);
        T dx[4], dp[4], pv[4], rv[4];
        to_rows(Dx, dx, lane);
        if (!last) {
#pragma unroll
          for (int ab = 0; ab < NB; ++ab)
#pragma unroll
            for (int kk = 0; kk < 4; ++kk) Dp = MT<T>::fma(pa[ab][kk], cf[g].bt(1, ab, jb, kk, lane), Dp);
          to_rows(Dp, dp, lane);
        }
#pragma unroll
        for (int m = 0; m < L::NR; ++m) {
          const int64_t row = row0 + L::row(m, lane);
          const bool ok = row < n;
          const int64_t off = row * K + cbase + jb * 16;
          T x[L::NC];
#pragma unroll
          for (int e = 0; e < L::NC; ++e) x[e] = xa[jb][m * L::NC + e] + dx[m * L::NC + e];  // X + P lambda
          if (ok) L::template store_p<NT>(X + off, x);
          T* pvm = pv + m * L::NC;
          T* rvm = rv + m * L::NC;
#pragma unroll
          for (int e = 0; e < L::NC; ++e) {
            rvm[e] = (ok && !last) ? ra[jb][m * L::NC + e] : T(0);
            pvm[e] = (ok && !last) ? rvm[e] + dp[m * L::NC + e] : T(0);  // R + P beta
          }
          if (ok && !last) L::store(Pm + off, pvm);
        }
        if (!last) {
          from_rows(pv, pn[jb], lane);
          from_rows(rv, rd[jb], lane);
        }
      }
      if (!last) gram_tiles<NB>(acc[g], pn, rd);  // rho = <<P_new, R>>
      if constexpr (PIPE)
#pragma unroll
        for (int jb = 0; jb < NB; ++jb)
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            pa[jb][e] = pnx[jb][e];
            xa[jb][e] = xnx[jb][e];
            ra[jb][e] = rnx[jb][e];
          }
    });
  }
  }
  finish_mfma<K, PW, false, perm_of<T>(), GW>(acc, G0, smem, part + (int64_t)blockIdx.x * pl.W, pl);
}

// ---------------------------------------------------------------- SpMM
// Element access at base + e. With O32 every byte offset into the operands
// fits in 32 bits, and the access is a uniform 64-bit base plus a 32-bit lane
// offset: one address operation per access instead of 64-bit arithmetic.
template <bool O32>
using EIdx = typename std::conditional<O32, uint32_t, int64_t>::type;
template <bool O32, typename V, typename E>
__device__ __forceinline__ V ld_at(const E* base, EIdx<O32> e) {
  if constexpr (O32)
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(base) + e * static_cast<uint32_t>(sizeof(E)));
  else
    return *reinterpret_cast<const V*>(base + e);
}
template <bool O32, typename V, typename E>
__device__ __forceinline__ void st_at(E* base, EIdx<O32> e, const V& v) {
  if constexpr (O32)
    *reinterpret_cast<V*>(reinterpret_cast<char*>(base) + e * static_cast<uint32_t>(sizeof(E))) = v;
  else
    *reinterpret_cast<V*>(base + e) = v;
}

// Q = A P with the partial alpha = <<P, Q>>. A wave takes steps of 8 rows of
// its column group, 8 lanes per row: lane l holds columns 2(l&7), 2(l&7)+1 of
// each 16-column block of row (l>>3) (16-byte gathers). One exchange between
// lanes l and l^8 (DPP row_ror:8; they hold rows 2s and 2s+1, s = l>>4) gives
// lane l column sigma(l&15) = 2(l&7) + ((l>>3)&1) of both rows: the operands
// of two 16x16x4 products (rows 2kc + v, kc = l>>4, v = 0, 1) whose result is
// the 8-row block product with rows and columns permuted by sigma.
//
// Software pipelined so that no wait on a younger load also waits for the
// current gathers (loads retire in issue order): per step the wave issues the
// gathers of step s, then the index chunk of the next step (CSR range loaded
// one step earlier), then the CSR range two steps ahead and the schedule
// entry three steps ahead, and only then consumes the gathers. All loads are
// unconditional (clamped rows and entries).
//
// SELL: the matrix is in sliced ELLPACK storage with slices of C = 16 step
// positions (Section 4 names SELL-C-sigma as the remedy for the product's
// cache behaviour). `rowptr` then holds the first slot of every slice, a
// slice of width w stores its two halves of 8 positions one after the other,
// each slot by slot: slot t of position 8 h + r of slice S sits at
// rowptr[S] + 8 w h + 8 t + r in `colind` and `vals` (value 0 in padding),
// and `pl.sched` maps positions to rows. A slice's width is the same for
// every lane of a step, so the index loads are coalesced (an 8-row step
// reads one contiguous run) and rows longer than 8 entries cost no
// divergent chunk loop.
__device__ __forceinline__ int dpp_ror8(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0x128, 0xF, 0xF, false);  // row_ror:8
}
__device__ __forceinline__ double dpp_ror8(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = dpp_ror8(static_cast<int>(v & 0xffffffffLL));
  const int hi = dpp_ror8(static_cast<int>(v >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}

// broadcast of lane `SRC` of each aligned group of 8 lanes (ds_swizzle bit
// mode: lane = (lane & 0x18) | SRC within 32)
template <int SRC>
__device__ __forceinline__ int bc8_i(int x) {
  return __builtin_amdgcn_ds_swizzle(x, (SRC << 5) | 0x18);
}
template <int SRC>
__device__ __forceinline__ double bc8(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = bc8_i<SRC>(static_cast<int>(v & 0xffffffffLL));
  const int hi = bc8_i<SRC>(static_cast<int>(v >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned int>(lo));
}
template <int SRC>
__device__ __forceinline__ float bc8(float x) {
  return __int_as_float(bc8_i<SRC>(__float_as_int(x)));
}

// CSR range and 8 (column, value) pairs of a lane's row
template <typename T>
struct Row8 {
  int j0, j1;
  int cols[8];
  T vs[8];
};

// lane cg of the row loads entry j + cg; entry u is then spread from lane u
template <typename T, int U = 0>
__device__ __forceinline__ void spread8(Row8<T>& r, int c, T v) {
  if constexpr (U < 8) {
    r.cols[U] = bc8_i<U>(c);
    r.vs[U] = bc8<U>(v);
    spread8<T, U + 1>(r, c, v);
  }
}

template <typename T, int K, int PW, bool O32, bool SELL>
__global__ __launch_bounds__(kBlock) void k_spmm_mfma(Plan pl, const int32_t* __restrict__ rowptr,
                                                      const int32_t* __restrict__ colind, const T* __restrict__ vals,
                                                      const T* __restrict__ Pm, T* __restrict__ Q,
                                                      double* __restrict__ part, const DevState* st) {
  if (halted(st)) return;
  using Gm = MGeo<K, PW>;
  using T2 = typename V2m<T>::type;
  constexpr int NB = Gm::NB;
  __shared__ double smem[smem_doubles<K, PW, 0>()];
  const int lane = threadIdx.x & 63, rr = lane >> 3, cg = lane & 7;
  const bool odd = (lane >> 3) & 1;
  const int64_t n = pl.n;
  const WaveWork ww = wave_work_sp<Gm::NG>((n + 7) / 8, pl.sp_chunk[0]);
  const int G = ww.group;
  const int c0 = G * PW + 2 * cg;
  MAcc<NB> acc;
  acc.zero();
  const int32_t* __restrict__ sched = pl.sched;
  using E = EIdx<O32>;
  auto row_of = [&](int64_t step) -> int {
    int64_t e = step * 8 + rr;
    e = e < n ? e : n - 1;
    return sched ? ld_at<O32, int32_t>(sched, static_cast<E>(e)) : static_cast<int>(e);
  };
  // entry range of this lane's row for `step` (SELL: address of the row's
  // slot 0 and the slice width; two steps of 8 positions share a slice)
  auto range = [&](int64_t step, int row, int& j0, int& j1) {
    if constexpr (SELL) {
      const E sl = static_cast<E>(step >> 1);
      const int b0 = ld_at<O32, int32_t>(rowptr, sl), b1 = ld_at<O32, int32_t>(rowptr, sl + 1);
      j1 = (b1 - b0) >> 4;
      j0 = b0 + 8 * j1 * static_cast<int>(step & 1) + rr;
    } else {
      j0 = ld_at<O32, int32_t>(rowptr, static_cast<E>(row));
      j1 = ld_at<O32, int32_t>(rowptr, static_cast<E>(row) + 1);
    }
  };
  // entry t0 + cg of the row (clamped into the row; the value of an entry
  // past its end is 0, so its product adds nothing)
  auto idx_load = [&](int j0, int j1, int t0, int& c, T& v) {
    if constexpr (SELL) {
      const int t = t0 + cg;
      const int jj = j0 + 8 * min(t, j1 - 1);
      c = ld_at<O32, int32_t>(colind, static_cast<E>(jj));
      const T x = ld_at<O32, T>(vals, static_cast<E>(jj));
      v = t < j1 ? x : T(0);
    } else {
      const int jj = max(min(j0 + t0 + cg, j1 - 1), 0);
      c = ld_at<O32, int32_t>(colind, static_cast<E>(jj));
      const T x = ld_at<O32, T>(vals, static_cast<E>(jj));
      v = j0 + t0 + cg < j1 ? x : T(0);
    }
  };
  const int64_t tw = ww.stride;
  const int64_t last = ww.end > ww.first ? ww.end - 1 : ww.first;
  int64_t s = ww.first;
  Row8<T> cur;
  int cur_row = 0, row1 = 0, row2 = 0;
  int nj0 = 0, nj1 = 0;  // CSR range of step s + tw
  if (s < ww.end) {
    cur_row = row_of(s);
    row1 = row_of(min(s + tw, last));
    row2 = row_of(min(s + 2 * tw, last));
    range(s, cur_row, cur.j0, cur.j1);
    range(min(s + tw, last), row1, nj0, nj1);
    int c;
    T v;
    idx_load(cur.j0, cur.j1, 0, c, v);
    spread8<T>(cur, c, v);
  }
  for (; s < ww.end; s += tw) {
    const bool ok = s * 8 + rr < n;
    const E i = static_cast<E>(cur_row);
    // 1. gathers of the current step (first block) and the own row of P
    T2 xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = ld_at<O32, T2>(Pm, static_cast<E>(cur.cols[u]) * K + c0);
    T2 pv[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) pv[b] = ld_at<O32, T2>(Pm, i * K + c0 + 16 * b);
    // 2. index chunk of the next step
    Row8<T> nxt;
    nxt.j0 = nj0;
    nxt.j1 = nj1;
    int nc;
    T nv;
    idx_load(nj0, nj1, 0, nc, nv);
    // 3. CSR range two steps ahead, schedule entry three steps ahead
    range(min(s + 2 * tw, last), row2, nj0, nj1);
    const int row3 = row_of(min(s + 3 * tw, last));
    // 4. consume the gathers, block by block
    T q[NB][2];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b > 0) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          xv[u] = ld_at<O32, T2>(Pm, static_cast<E>(cur.cols[u]) * K + c0 + 16 * b);
      }
      T q0 = T(0), q1 = T(0);
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        q0 = fma(cur.vs[u], xv[u].x, q0);
        q1 = fma(cur.vs[u], xv[u].y, q1);
      }
      q[b][0] = q0;
      q[b][1] = q1;
    }
    // rows with more than 8 entries: remaining chunks without pipelining
    for (int t0 = 8; SELL ? t0 < cur.j1 : cur.j0 + t0 < cur.j1; t0 += 8) {
      Row8<T> ex;
      int c;
      T v;
      idx_load(cur.j0, cur.j1, t0, c, v);
      spread8<T>(ex, c, v);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          xv[u] = ld_at<O32, T2>(Pm, static_cast<E>(ex.cols[u]) * K + c0 + 16 * b);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          q[b][0] = fma(ex.vs[u], xv[u].x, q[b][0]);
          q[b][1] = fma(ex.vs[u], xv[u].y, q[b][1]);
        }
      }
    }
    // store Q; exchange P and Q values between lanes l and l^8
    double pe[NB][2], qe[NB][2];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (ok) st_at<O32>(Q, i * K + c0 + 16 * b, T2{q[b][0], q[b][1]});
      const double p0 = ok ? static_cast<double>(pv[b].x) : 0.0, p1 = ok ? static_cast<double>(pv[b].y) : 0.0;
      const double q0 = ok ? static_cast<double>(q[b][0]) : 0.0, q1 = ok ? static_cast<double>(q[b][1]) : 0.0;
      const double pr = dpp_ror8(odd ? p0 : p1), qr = dpp_ror8(odd ? q0 : q1);
      pe[b][0] = odd ? pr : p0;
      pe[b][1] = odd ? p1 : pr;
      qe[b][0] = odd ? qr : q0;
      qe[b][1] = odd ? q1 : qr;
    }
    // alpha = <<P, Q>> over the 8 rows (sigma-permuted)
#pragma unroll
    for (int ab = 0; ab < NB; ++ab)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int v = 0; v < 2; ++v) acc.g[ab * NB + jb] = mfma(pe[ab][v], qe[jb][v], acc.g[ab * NB + jb]);
    spread8<T>(nxt, nc, nv);
    cur = nxt;
    cur_row = row1;
    row1 = row2;
    row2 = row3;
  }
  finish_mfma<K, PW, false>(acc, G, smem, part + (int64_t)blockIdx.x * pl.W, pl);
}

// FP32 variant: 4 lanes per row and 16 rows per step, lane l holding columns
// 4(l&3)..4(l&3)+3 of each block of row (l>>2) (16-byte gathers). The (column,
// value) pairs of a row are loaded two per lane and broadcast within the quad
// (DPP quad_perm). A 4 x 4 transpose among lanes l, l^4, l^8, l^12 (three XOR
// swizzles) gives lane l column tau(l&15) = 4(l&3) + ((l>>2)&3) of rows
// 4s + m (s = l>>4, m = 0..3): the operands of four 16x16x4 products.
template <int I>
__device__ __forceinline__ int quad_bcast(int x) {
  return __builtin_amdgcn_mov_dpp(x, I * 0x55, 0xF, 0xF, false);  // quad_perm [I,I,I,I]
}
template <int I>
__device__ __forceinline__ float quad_bcast(float x) {
  return __int_as_float(quad_bcast<I>(__float_as_int(x)));
}
// in v[e] = X[row t][e], out w[m] = X[row m][t] as FP64 operands
__device__ __forceinline__ void transpose4(const float (&v)[4], double (&w)[4], int t) {
  float f[4];
  transpose4(v, f, t);
#pragma unroll
  for (int m = 0; m < 4; ++m) w[m] = static_cast<double>(f[m]);
}

struct Row8f {
  int j0, j1;
  int cols[8];
  float vs[8];
};

template <int U = 0>
__device__ __forceinline__ void spread_quad(Row8f& r, const int (&c)[2], const float (&v)[2]) {
  if constexpr (U < 8) {
    r.cols[U] = quad_bcast<U & 3>(c[U >> 2]);
    r.vs[U] = quad_bcast<U & 3>(v[U >> 2]);
    spread_quad<U + 1>(r, c, v);
  }
}

template <int K, int PW, bool O32, bool SELL>
__global__ __launch_bounds__(kBlock) void k_spmm_mfma_f32(Plan pl, const int32_t* __restrict__ rowptr,
                                                          const int32_t* __restrict__ colind,
                                                          const float* __restrict__ vals, const float* __restrict__ Pm,
                                                          float* __restrict__ Q, double* __restrict__ part,
                                                          const DevState* st) {
  if (halted(st)) return;
  using Gm = MGeo<K, PW>;
  constexpr int NB = Gm::NB;
  __shared__ double smem[smem_doubles<K, PW, 0>()];
  const int lane = threadIdx.x & 63, rr = lane >> 2, cq = lane & 3, tq = (lane >> 2) & 3;
  const int64_t n = pl.n;
  const WaveWork ww = wave_work_sp<Gm::NG>((n + 15) / 16, pl.sp_chunk[1]);
  const int G = ww.group;
  const int c0 = G * PW + 4 * cq;
  MAcc<NB> acc;
  acc.zero();
  const int32_t* __restrict__ sched = pl.sched;
  using E = EIdx<O32>;
  auto row_of = [&](int64_t step) -> int {
    int64_t e = step * 16 + rr;
    e = e < n ? e : n - 1;
    return sched ? ld_at<O32, int32_t>(sched, static_cast<E>(e)) : static_cast<int>(e);
  };
  // entry range of this lane's row for `step` (SELL: address of the row's
  // slot 0 and the slice width; one step per slice)
  auto range = [&](int64_t step, int row, int& j0, int& j1) {
    if constexpr (SELL) {
      const int b0 = ld_at<O32, int32_t>(rowptr, static_cast<E>(step)),
                b1 = ld_at<O32, int32_t>(rowptr, static_cast<E>(step) + 1);
      j1 = (b1 - b0) >> 4;
      j0 = b0 + 8 * j1 * (rr >> 3) + (rr & 7);
    } else {
      j0 = ld_at<O32, int32_t>(rowptr, static_cast<E>(row));
      j1 = ld_at<O32, int32_t>(rowptr, static_cast<E>(row) + 1);
    }
  };
  // entries t0 + cq and t0 + cq + 4 of the row (clamped into the row; past
  // its end the value is 0, so the product adds nothing)
  auto idx_load = [&](int j0, int j1, int t0, int (&c)[2], float (&v)[2]) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int t = t0 + cq + 4 * h;
      const int jj = SELL ? j0 + 8 * min(t, j1 - 1) : max(min(j0 + t, j1 - 1), 0);
      c[h] = ld_at<O32, int32_t>(colind, static_cast<E>(jj));
      const float x = ld_at<O32, float>(vals, static_cast<E>(jj));
      v[h] = (SELL ? t < j1 : j0 + t < j1) ? x : 0.f;
    }
  };
  const int64_t tw = ww.stride;
  const int64_t last = ww.end > ww.first ? ww.end - 1 : ww.first;
  int64_t s = ww.first;
  Row8f cur;
  int cur_row = 0, row1 = 0, row2 = 0;
  int nj0 = 0, nj1 = 0;
  if (s < ww.end) {
    cur_row = row_of(s);
    row1 = row_of(min(s + tw, last));
    row2 = row_of(min(s + 2 * tw, last));
    range(s, cur_row, cur.j0, cur.j1);
    range(min(s + tw, last), row1, nj0, nj1);
    int c[2];
    float v[2];
    idx_load(cur.j0, cur.j1, 0, c, v);
    spread_quad(cur, c, v);
  }
  for (; s < ww.end; s += tw) {
    const bool ok = s * 16 + rr < n;
    const E i = static_cast<E>(cur_row);
    float4 xv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) xv[u] = ld_at<O32, float4>(Pm, static_cast<E>(cur.cols[u]) * K + c0);
    // two-block groups: the second block's gathers go out with the first's
    // (wider groups reload per block to stay within the registers)
    constexpr bool UP = NB == 2;
    float4 xw[UP ? 8 : 1];
    if constexpr (UP) {
#pragma unroll
      for (int u = 0; u < 8; ++u) xw[u] = ld_at<O32, float4>(Pm, static_cast<E>(cur.cols[u]) * K + c0 + 16);
    }
    float4 pv[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) pv[b] = ld_at<O32, float4>(Pm, i * K + c0 + 16 * b);
    Row8f nxt;
    nxt.j0 = nj0;
    nxt.j1 = nj1;
    int nc[2];
    float nv[2];
    idx_load(nj0, nj1, 0, nc, nv);
    range(min(s + 2 * tw, last), row2, nj0, nj1);
    const int row3 = row_of(min(s + 3 * tw, last));
    float q[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (b > 0) {
        if constexpr (UP) {
#pragma unroll
          for (int u = 0; u < 8; ++u) xv[u] = xw[u];
        } else {
#pragma unroll
          for (int u = 0; u < 8; ++u)
            xv[u] = ld_at<O32, float4>(Pm, static_cast<E>(cur.cols[u]) * K + c0 + 16 * b);
        }
      }
      float a[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const float x[4] = {xv[u].x, xv[u].y, xv[u].z, xv[u].w};
#pragma unroll
        for (int e = 0; e < 4; ++e) a[e] = fmaf(cur.vs[u], x[e], a[e]);
      }
#pragma unroll
      for (int e = 0; e < 4; ++e) q[b][e] = a[e];
    }
    for (int t0 = 8; SELL ? t0 < cur.j1 : cur.j0 + t0 < cur.j1; t0 += 8) {
      Row8f ex;
      int c[2];
      float v[2];
      idx_load(cur.j0, cur.j1, t0, c, v);
      spread_quad(ex, c, v);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
          xv[u] = ld_at<O32, float4>(Pm, static_cast<E>(ex.cols[u]) * K + c0 + 16 * b);
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const float x[4] = {xv[u].x, xv[u].y, xv[u].z, xv[u].w};
#pragma unroll
          for (int e = 0; e < 4; ++e) q[b][e] = fmaf(ex.vs[u], x[e], q[b][e]);
        }
      }
    }
    double pt[NB][4], qt[NB][4];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      if (ok) st_at<O32>(Q, i * K + c0 + 16 * b, float4{q[b][0], q[b][1], q[b][2], q[b][3]});
      const float pz[4] = {ok ? pv[b].x : 0.f, ok ? pv[b].y : 0.f, ok ? pv[b].z : 0.f, ok ? pv[b].w : 0.f};
      const float qz[4] = {ok ? q[b][0] : 0.f, ok ? q[b][1] : 0.f, ok ? q[b][2] : 0.f, ok ? q[b][3] : 0.f};
      transpose4(pz, pt[b], tq);
      transpose4(qz, qt[b], tq);
    }
    // alpha = <<P, Q>> over the 16 rows (tau-ordered)
#pragma unroll
    for (int ab = 0; ab < NB; ++ab)
#pragma unroll
      for (int jb = 0; jb < NB; ++jb)
#pragma unroll
        for (int m = 0; m < 4; ++m) acc.g[ab * NB + jb] = mfma(pt[ab][m], qt[jb][m], acc.g[ab * NB + jb]);
    spread_quad(nxt, nc, nv);
    cur = nxt;
    cur_row = row1;
    row1 = row2;
    row2 = row3;
  }
  finish_mfma<K, PW, false, Perm::tau>(acc, G, smem, part + (int64_t)blockIdx.x * pl.W, pl);
}

int env_set(const char* name) {
  const char* v = std::getenv(name);
  return v != nullptr && v[0] != '\0' && v[0] != '0';
}

template <typename F>
bool dispatch_mfma_w(int k, int w, F&& f) {
  if (!w) return false;
  auto withK = [&](auto Kc) -> bool {
    constexpr int K = decltype(Kc)::value;
    if (w == 16) {
      f(Kc, std::integral_constant<int, 16>());
      return true;
    }
    if constexpr (K % 32 == 0)
      if (w == 32) {
        f(Kc, std::integral_constant<int, 32>());
        return true;
      }
    if constexpr (K == 64)
      if (w == 64) {
        f(Kc, std::integral_constant<int, 64>());
        return true;
      }
    return false;
  };
  switch (k) {
    case 16: return withK(std::integral_constant<int, 16>());
    case 32: return withK(std::integral_constant<int, 32>());
    case 48: return withK(std::integral_constant<int, 48>());
    case 64: return withK(std::integral_constant<int, 64>());
    case 80: return withK(std::integral_constant<int, 80>());
    case 96: return withK(std::integral_constant<int, 96>());
    case 112: return withK(std::integral_constant<int, 112>());
    case 128: return withK(std::integral_constant<int, 128>());
    default: return false;
  }
}

// the launch must give every XCD (or the whole grid below 8 workgroups) at
// least one wave per column group
template <typename F>
bool dispatch_mfma(const Plan& pl, F&& f) {
  return dispatch_mfma_w(pl.k, pl.mfma, f);
}

void check_grid(const Plan& pl, int w) {
  const int ng = pl.k / w;
  const int min_waves = pl.nwg < 8 ? pl.nwg * 4 : (pl.nwg / 8) * 4;
  if (min_waves < ng) throw std::runtime_error("matrix-core launch: fewer waves than column groups");
}

}  // namespace

// The sparse product takes groups of 32 columns where k allows (p then
// divides 32, and each group's p x p Gram blocks lie on the diagonal of its
// 32 x 32 product): one wave gathers both 16-column halves of a row with one
// set of index loads, where two waves of 16 columns each load them twice.
// Measured 5-24 % faster for k = 32..128.
int mfma_sp_width(int k, int w, int p) {
  if (w == 16 && k % 32 == 0 && 32 % p == 0 && !env_set("BCG_SP_W16")) return 32;
  return w;
}

int mfma_width(int64_t nnz, int k, int p) {
  if (env_set("BCG_NO_MFMA") || env_set("BCG_GENERIC_ONLY") || nnz < 1) return 0;
  if (k % 16 != 0 || k > 128) return 0;
  if (p <= 16 && 16 % p == 0) return 16;
  if (p == 32 && k % 32 == 0) return 32;
  if (p == 64 && k == 64) return 64;
  return 0;
}

void mfma_sp_grid(Plan& pl) {
  const int w = pl.sp_w, ng = pl.k / w;
  const bool share = ng <= 4 && 4 % ng == 0;
  const int ngb = share ? 1 : (ng + 3) / 4, wpg = share ? 4 / ng : 1;
  const int kwg = share ? pl.k : 4 * w;  // columns one workgroup covers
  for (int prec = 0; prec < 2; ++prec) {
    const int rows_step = prec ? 16 : 8, elem = prec ? 4 : 8;
    const int64_t nsteps = (pl.n + rows_step - 1) / rows_step;
    // steps per wave: a power of two (chunks that straddle the rows and
    // planes of a tiled stencil order measure up to 1.7x slower), covering
    // at least 1024 rows per workgroup (one 32 x 32 tile plane), and large
    // enough that a workgroup's partial row (8 W bytes) stays below 1/32 of
    // the bytes its chunk moves
    const double step_bytes = static_cast<double>(wpg) * rows_step * (2.0 * kwg * elem + 12.0);
    const int need = std::max(static_cast<int>(std::ceil(256.0 * pl.W / step_bytes)), 1024 / (wpg * rows_step));
    int chunk = 1;
    while (chunk < need) chunk *= 2;
    if (const char* e = std::getenv("BCG_SP_CHUNK")) {  // override (a power of two)
      const int v = std::atoi(e);
      if (v > 0 && (v & (v - 1)) == 0) chunk = v;
    }
    const int64_t per = (nsteps + 7) / 8;
    int64_t span = static_cast<int64_t>(chunk) * wpg, nch = (per + span - 1) / span;
    while (8 * ngb * nch > kMaxSpWG) {
      chunk *= 2;
      span = static_cast<int64_t>(chunk) * wpg;
      nch = (per + span - 1) / span;
    }
    pl.sp_chunk[prec] = chunk;
    pl.sp_nwg[prec] = static_cast<int>(8 * ngb * nch);
    // 32-bit byte offsets when the vectors, the entries and the row pointers
    // all stay below 4 GiB (BCG_WIDE_OFFSETS forces 64-bit offsets)
    const int64_t lim = int64_t(1) << 32;
    pl.sp_o32[prec] = pl.n * pl.k * elem < lim && pl.nnz * elem < lim && (pl.n + 1) * 4 < lim &&
                      !env_set("BCG_WIDE_OFFSETS");
    // non-temporal streams in the update passes when X, R, P, Q and A
    // together exceed the 256 MiB memory-side cache
    const int64_t working = 4 * pl.n * pl.k * elem + pl.nnz * (elem + 4) + 4 * (pl.n + 1);
    pl.nt[prec] = working > (int64_t(256) << 20);
    // column groups per wave of the update passes: a whole 128-byte line of
    // every row where one 16-column FP32 group covers only half of one (both
    // groups then move in whole-line instructions; BCG_UPDATE_GW = 1 or 2
    // overrides for 16-column groups)
    const int ng = pl.mfma > 0 ? pl.k / pl.mfma : 1;
    int gw = (prec == 1 && pl.mfma == 16 && ng % 2 == 0) ? 2 : 1;
    if (const char* e = std::getenv("BCG_UPDATE_GW")) {
      const int v = std::atoi(e);
      if ((v == 1 || v == 2) && ng % v == 0 && (v == 1 || pl.mfma == 16)) gw = v;
    }
    pl.ugw[prec] = gw;
    // vector update passes beside the matrix-core sparse product where they
    // measured faster on the 256^3, k = 128 Poisson workload: the FP32 X/P
    // pass for p <= 16 (9.1 against 9.6 ms at p = 16, 8.0 against 9.2 ms at
    // p = 8), the FP32 R update for p <= 8 (5.0 against 5.4 ms at p = 8; at
    // p = 16 the vector one takes 7.6 against 5.3 ms), the FP64 R update for
    // p <= 16 (9.5 against 10.4 ms at p = 16); k = 16 is faster on the matrix
    // cores throughout. BCG_UPDATE_VEC32 / BCG_UPDATE_VEC64 = 0..3 override
    // (bit 0: R update, bit 1: X/P pass).
    int vec = 0;
    if (pl.fast && pl.k == 128) vec = prec ? (pl.p <= 8 ? 3 : 2) : 1;
    if (const char* e = std::getenv(prec ? "BCG_UPDATE_VEC32" : "BCG_UPDATE_VEC64")) {
      const int v = std::atoi(e);
      if (v >= 0 && v <= 3) vec = pl.fast ? v : 0;
    }
    pl.upd_vec[prec] = vec;
  }
}

int mfma_grid(int64_t n, int k, int w) {
  const int64_t ng = k / w;
  const int64_t units = ((n + 15) / 16) * ng;
  int64_t nwg = (units + 3) / 4;
  if (nwg > kMaxWG) nwg = kMaxWG;
  if (nwg < 1) nwg = 1;
  if (ng > 4) {
    if (nwg < 2) nwg = 2;
    if (nwg >= 8 && nwg < 16) nwg = 7;
  }
  return static_cast<int>(nwg);
}

template <typename T>
void launch_spmm_mfma(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const T* vals, const T* P, T* Q,
                      double* part, const DevState* st, hipStream_t s) {
  const int prec = std::is_same<T, float>::value ? 1 : 0;
  if (pl.sp_chunk[prec] == 0) check_grid(pl, pl.sp_w);
  const dim3 grid(pl.sp_nwg[prec]);
  const int mode = (pl.sp_o32[prec] != 0 ? 1 : 0) | (pl.sell ? 2 : 0);
  dispatch_mfma_w(pl.k, pl.sp_w, [&](auto Kc, auto Wc) {
    constexpr int K = decltype(Kc)::value, W = decltype(Wc)::value;
    auto go = [&](auto O32c, auto SELLc) {
      constexpr bool O32 = decltype(O32c)::value, SELL = decltype(SELLc)::value;
      if constexpr (std::is_same<T, float>::value)
        hipLaunchKernelGGL((k_spmm_mfma_f32<K, W, O32, SELL>), grid, dim3(kBlock), 0, s, pl, rowptr, colind, vals, P,
                           Q, part, st);
      else
        hipLaunchKernelGGL((k_spmm_mfma<T, K, W, O32, SELL>), grid, dim3(kBlock), 0, s, pl, rowptr, colind, vals, P,
                           Q, part, st);
    };
    using t_ = std::true_type;
    using f_ = std::false_type;
    switch (mode) {
      case 0: go(f_(), f_()); break;
      case 1: go(t_(), f_()); break;
      case 2: go(f_(), t_()); break;
      default: go(t_(), t_()); break;
    }
  });
}

template <typename F>
void with_gw(int gw, F&& f) {
  if (gw == 2)
    f(std::integral_constant<int, 2>());
  else
    f(std::integral_constant<int, 1>());
}

template <typename T>
void launch_update_r_mfma(const Plan& pl, T* R, const T* Q, const T* lam, double* part, const DevState* st,
                          hipStream_t s) {
  check_grid(pl, pl.mfma);
  const bool nt = pl.nt[std::is_same<T, float>::value ? 1 : 0] != 0;
  dispatch_mfma(pl, [&](auto Kc, auto Wc) {
    constexpr int K = decltype(Kc)::value, W = decltype(Wc)::value;
    with_gw(pl.ugw[std::is_same<T, float>::value ? 1 : 0], [&](auto Gc) {
      constexpr int GW = (MGeo<K, W>::NG % decltype(Gc)::value == 0 && (decltype(Gc)::value == 1 || W == 16))
                             ? decltype(Gc)::value
                             : 1;
      if (stream_nt<T, K, W, GW>() && nt)
        hipLaunchKernelGGL((k_update_r_mfma<T, K, W, stream_nt<T, K, W, GW>(), GW>), dim3(pl.nwg), dim3(kBlock), 0, s,
                           pl, R, Q, lam, part, st);
      else
        hipLaunchKernelGGL((k_update_r_mfma<T, K, W, false, GW>), dim3(pl.nwg), dim3(kBlock), 0, s, pl, R, Q, lam,
                           part, st);
    });
  });
}

template <typename T>
void launch_update_xp_mfma(const Plan& pl, T* X, T* P, const T* R, const T* lam, const T* beta, double* part,
                           const DevState* st, hipStream_t s) {
  check_grid(pl, pl.mfma);
  const bool nt = pl.nt[std::is_same<T, float>::value ? 1 : 0] != 0;
  dispatch_mfma(pl, [&](auto Kc, auto Wc) {
    constexpr int K = decltype(Kc)::value, W = decltype(Wc)::value;
    with_gw(pl.ugw[std::is_same<T, float>::value ? 1 : 0], [&](auto Gc) {
      constexpr int GW = (MGeo<K, W>::NG % decltype(Gc)::value == 0 && (decltype(Gc)::value == 1 || W == 16))
                             ? decltype(Gc)::value
                             : 1;
      if (stream_nt<T, K, W, GW>() && nt)
        hipLaunchKernelGGL((k_update_xp_mfma<T, K, W, stream_nt<T, K, W, GW>(), GW>), dim3(pl.nwg), dim3(kBlock), 0,
                           s, pl, X, P, R, lam, beta, part, st);
      else
        hipLaunchKernelGGL((k_update_xp_mfma<T, K, W, false, GW>), dim3(pl.nwg), dim3(kBlock), 0, s, pl, X, P, R, lam,
                           beta, part, st);
    });
  });
}

#define BCG_MFMA_INST(T)                                                                                           \
  template void launch_spmm_mfma<T>(const Plan&, const int32_t*, const int32_t*, const T*, const T*, T*, double*, \
                                    const DevState*, hipStream_t);                                                 \
  template void launch_update_r_mfma<T>(const Plan&, T*, const T*, const T*, double*, const DevState*,            \
                                        hipStream_t);                                                              \
  template void launch_update_xp_mfma<T>(const Plan&, T*, T*, const T*, const T*, const T*, double*,              \
                                         const DevState*, hipStream_t);
BCG_MFMA_INST(double)
BCG_MFMA_INST(float)

}  // namespace bcg
