// Internal declarations shared by the block CG kernels and the solver runtime.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bcg {

constexpr int kBlock = 256;        // threads per workgroup of the row kernels
constexpr int kTileElems = 1024;   // rows*k elements staged per LDS tile
constexpr int kMaxWG = 1024;       // cap on workgroups of the row kernels
constexpr int kMaxSpWG = 16384;    // cap on workgroups of the chunked sparse product
constexpr int kRedSplits = 64;     // first-stage row splits of a reduction over many rows
constexpr int kRedSplitRows = 2048;  // reductions over more rows take two stages
constexpr int kNabMax = 8;         // entry blocks per thread in fused products
constexpr int kLamLds = 2048;      // coefficient entries kept in LDS

// Device-side solve state. Every per-iteration kernel returns at entry once
// `done` is set. `last` marks the final iteration (stop rule met, iteration
// cap, breakdown after the residual update): its X/P pass then applies only
// X += P lambda; the sparse product after it returns at entry and the
// reduction after that sets `done`.
struct DevState {
  int done;
  int status;
  int iter;
  int last;
  unsigned int ticket;  // workgroups of a reduce-and-solve launch that have finished (0 between launches)
  double max_ratio;     // largest column ratio ||R_j|| / r0_j after the last iteration
};

// Entry test of the sparse products: nothing is left to do once the final
// iteration has been marked.
__device__ __forceinline__ bool halted(const DevState* st) {
  return st != nullptr && (*reinterpret_cast<const volatile int*>(&st->done) != 0 ||
                           *reinterpret_cast<const volatile int*>(&st->last) != 0);
}

// Geometry of one solve: the subalgebra, the packed product layout and the
// thread plan of the block-product accumulation.
struct Plan {
  int64_t n;
  int64_t nnz;
  int k, p, q;
  int qo;       // packed blocks: 1 for the global subalgebra, q otherwise
  int global;   // 1: product summed over the q groups
  int dec;      // 1: p = 1 with independent columns (zero lanes allowed)
  int E;        // qo * p * p packed product entries
  int W;        // partial row width = E + k (product | column norms)
  int rb;       // register block of the product accumulation (1 or 2)
  int pb;       // p / rb
  int EB;       // entry blocks = qo * pb * pb
  int S;        // row slices when EB < kBlock
  int nab;      // entry blocks per thread when EB > kBlock
  int fused;    // 1: product accumulated inside the producing kernel
  int TR;       // rows per LDS tile
  int64_t ntiles;
  int nwg;      // workgroups of the row kernels
  int fast;     // 1: the k-specialised row kernels apply (k in {8..128}, p <= 16)
  int mfma;     // column-group width of the matrix-core row kernels (0: not used)
  int sp_w;     // column-group width of the matrix-core sparse product
  // sparse product of the matrix-core path, per precision (0: FP64, 1: FP32):
  // workgroups and steps per wave of its chunked grid (0 steps: persistent
  // grid of nwg workgroups)
  int sp_nwg[2];
  int sp_chunk[2];
  int sp_o32[2];  // sparse product with 32-bit lane offsets (FP64, FP32)
  int nt[2];      // row kernels stream dead operands non-temporally (FP64, FP32)
  int ugw[2];     // column groups per wave of the matrix-core update passes (FP64, FP32)
  // matrix-core plan whose R update (bit 0) / X-P pass (bit 1) run on the
  // k-specialised vector kernels instead (FP64, FP32)
  int upd_vec[2];
  const int32_t* sched;  // processing order of the sparse-product rows (nullptr: natural)
  int sell;     // 1: the matrix-core sparse product reads SELL-16-sigma storage
                // (rowptr: slice starts, sched: position -> row)
};

Plan make_plan(int64_t n, int64_t nnz, int k, int p, int global, int dec);
bool fast_supported(const Plan& pl);
// matrix-core row kernels: group width for (nnz, k, p), 0 where they do not
// apply; workgroup count that gives every XCD a wave per column group
int mfma_width(int64_t nnz, int k, int p);
// matrix-core sparse-product group width for row-kernel width w
int mfma_sp_width(int k, int w, int p);
int mfma_grid(int64_t n, int k, int w);
// chunked sparse-product grid of the matrix-core path (sets sp_nwg, sp_chunk)
void mfma_sp_grid(Plan& pl);

// ---- launchers (all enqueue on `s`; none synchronises) ----
// R = B - A X; norms partial; if with_p: P = R and <<R,R>> partial.
void launch_residual(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const double* vals,
                     const double* B, const double* X, double* R, double* P, double* part,
                     int with_p, hipStream_t s);
// FP32 inner start: s = max_j sqrt(norms_j); R32 = R64/s; P32 = R32; D32 = 0;
// <<R32,R32>> partial (FP64 accumulation) and norms partial.
void launch_cast_init(const Plan& pl, const double* R64, const double* norms, float* R32, float* P32,
                      float* D32, double* scale, double* part, hipStream_t s, double pfac = 0.0);
template <typename T>
void launch_spmm_product(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const T* vals,
                         const T* P, T* Q, double* part, const DevState* st, hipStream_t s);
template <typename T>
void launch_update_r(const Plan& pl, T* R, const T* Q, const T* lam, double* part, const DevState* st,
                     hipStream_t s);
template <typename T>
void launch_update_xp(const Plan& pl, T* X, T* P, const T* R, const T* lam, const T* beta, double* part,
                      const DevState* st, hipStream_t s);
// stand-alone product for plans whose products do not fit the fused path
template <typename T>
void launch_product(const Plan& pl, const T* X, const T* Y, double* part, const DevState* st, hipStream_t s);
// rows: partial rows to sum (-1: nwg); more than kRedSplitRows rows are
// summed in two stages through `scratch` (kRedSplits rows of width W).
void launch_reduce(const Plan& pl, const double* part, double* out, int width, DevState* st, hipStream_t s,
                   int rows = -1, double* scratch = nullptr);
// p x p solves of p in {2, 4, 8, 16, 32} run in registers, one wave per group;
// only those are fused into the reduction that produces their operands.
bool register_solve(int p);
// Lines 6-7: alpha = <<P, AP>> (partials of a_rows rows; more than
// kRedSplitRows go through `scratch` first) and, for r_rows > 0, rho =
// <<P, R>> of the previous X/P pass reduced; then lambda. A marked final
// iteration sets `done` here instead. For register_solve(p) one launch: its
// last workgroup to finish solves.
void launch_reduce_lambda(const Plan& pl, const double* partA, int a_rows, double* scratch, const double* partR,
                          int r_rows, double* alpha, double* rho, double* lam, float* lam32, double* ws, DevState* st,
                          hipStream_t s);
// Line 11 sums (<<R, R>> and the column norms, `rows` partial rows), then the
// stop rule and beta (line 12); for register_solve(p) one launch whose last
// workgroup to finish decides and solves.
void launch_reduce_beta(const Plan& pl, const double* partN, int rows, double* red_new, const double* r0,
                        const double* rho_old, double* beta, float* beta32, double* ws, double* ratios, DevState* st,
                        double tol, int it, int maxit, hipStream_t s);
// Stand-alone lambda solve, and stop rule with beta, from reduced operands:
// workgroup Gauss-Jordan for p <= 64, LDS / global-workspace kernels beyond.
void launch_solve_lambda(const Plan& pl, const double* alpha, const double* rho, double* lam, float* lam32,
                         double* ws, DevState* st, hipStream_t s);
void launch_conv_beta(const Plan& pl, const double* red_new, const double* r0, const double* rho_old,
                      double* beta, float* beta32, double* ws, double* ratios, DevState* st, double tol,
                      int it, int maxit, hipStream_t s);
void launch_axpy_scaled(int64_t count, double* X, const float* D, const double* scale, hipStream_t s);
// x *= c (count entries)
void launch_scale_vec(double* x, int64_t count, double c, hipStream_t s);
void launch_sampled_outer(int64_t n, int k, const int32_t* rowptr, const int32_t* colind, const double* Y,
                          const double* X, double alpha, double* out, hipStream_t s);
void launch_cast_values(int64_t nnz, const double* v, float* v32, hipStream_t s);
// values of SELL storage: slot e takes entry map[e] of v / v32 (0 where
// map[e] < 0, the padding)
void launch_sell_values(int64_t slots, const int32_t* map, const double* v, const float* v32, double* sv,
                        float* sv32, hipStream_t s);
void launch_check_perm(const int32_t* order, int64_t n, int* seen, int* flag, hipStream_t s);
void launch_check_csr(const int32_t* rowptr, const int32_t* colind, int64_t n, int64_t nnz, int* flag,
                      hipStream_t s);
// k-specialised row kernels (16-byte aligned block vectors; see fast_supported)
// R = B - A X with the column norms (with_p: also P = R and, when fused, the
// partial <<R, R>>); false when the plan has no k-specialised kernels
bool launch_residual_fast(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const double* vals,
                          const double* B, const double* X, double* R, double* P, double* part, int with_p,
                          hipStream_t s);
// FP32 start of a refinement step (see launch_cast_init); false when the plan
// has no k-specialised kernels
bool launch_cast_init_fast(const Plan& pl, const double* R64, const double* norms, float* R32, float* P32,
                           float* D32, double* scale, double* part, hipStream_t s, double pfac);
template <typename T>
void launch_spmm_fast(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const T* vals, const T* P,
                      T* Q, double* part, const DevState* st, hipStream_t s);
template <typename T>
void launch_update_r_fast(const Plan& pl, T* R, const T* Q, const T* lam, double* part, const DevState* st,
                          hipStream_t s);
template <typename T>
void launch_update_xp_fast(const Plan& pl, T* X, T* P, const T* R, const T* lam, const T* beta, double* part,
                           const DevState* st, hipStream_t s);

// matrix-core row kernels (k a multiple of 16; see mfma_width)
template <typename T>
void launch_spmm_mfma(const Plan& pl, const int32_t* rowptr, const int32_t* colind, const T* vals, const T* P,
                      T* Q, double* part, const DevState* st, hipStream_t s);
template <typename T>
void launch_update_r_mfma(const Plan& pl, T* R, const T* Q, const T* lam, double* part, const DevState* st,
                          hipStream_t s);
template <typename T>
void launch_update_xp_mfma(const Plan& pl, T* X, T* P, const T* R, const T* lam, const T* beta, double* part,
                           const DevState* st, hipStream_t s);

}  // namespace bcg
