// Solver runtime behind the C ABI: handle, workspace, the iteration driver of
// Algorithm 1 (Section 3, M = I) and the FP32/FP64 refinement loop.
//
// The host enqueues iterations in chunks and never waits inside a chunk: the
// kernels of every iteration return at entry once the device-side `done`
// flag is set (converged, breakdown or iteration cap), so the stop iteration
// is exactly the one the stop rule accepted. The host keeps two chunks in
// flight and reads the flag of the older one through pinned memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/bcg.h"
#include "bcg_internal.h"
#include "bcg_scale.h"

using namespace bcg;

namespace {

thread_local std::string g_error;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) return fail(BCG_EHIP, "%s: %s", #expr, hipGetErrorString(e_));    \
  } while (0)

struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <typename T>
int dalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(BCG_ENOMEM, "device allocation of %zu bytes failed", count * sizeof(T));
  }
  return BCG_OK;
}

// Row kernels of a solve: matrix-core kernels where the plan allows them,
// else the k-specialised kernels, else the generic ones. The first two access
// X two elements at a time and need it 16-byte aligned.
enum class RowPath { generic, fast, mfma };

RowPath row_path(const Plan& pl, bool x_aligned) {
  if (!x_aligned) return RowPath::generic;
  if (pl.mfma) return RowPath::mfma;
  if (pl.fast) return RowPath::fast;
  return RowPath::generic;
}

// Buffers of one precision's iteration: block vectors and coefficients.
template <typename T>
struct IterBuffers {
  const T* vals;
  T *X, *R, *P, *Q;
  const T *lam, *beta;
};

}  // namespace

struct bcg_handle {
  int device = 0;
  hipStream_t stream = nullptr;
  int64_t n = 0, nnz = 0;
  int k = 0, p = 0, variant = 0;
  Plan pl{};
  int32_t *rowptr = nullptr, *colind = nullptr;
  double* vals = nullptr;
  float* vals32 = nullptr;
  double *R = nullptr, *P = nullptr, *Q = nullptr;
  double *partA = nullptr, *partR = nullptr, *partN = nullptr;
  double* part2 = nullptr;  // first-stage rows of reductions over many partial rows
  double *alpha = nullptr, *rho = nullptr, *rnew = nullptr;
  double *lam = nullptr, *beta = nullptr, *ws = nullptr;
  float *lam32 = nullptr, *beta32 = nullptr;
  double *r0 = nullptr, *ratios = nullptr, *scale = nullptr;
  int32_t* sched = nullptr;  // optional row order of the sparse product
  // SELL-16-sigma copy of the matrix for the matrix-core sparse product
  int sell = 0, sell_sigma = 1;
  int64_t sell_slots = 0;
  int32_t *sl_ptr = nullptr, *sl_perm = nullptr, *sl_col = nullptr, *sl_map = nullptr;
  double* sl_val = nullptr;
  float* sl_val32 = nullptr;
  Plan pl_sell{};  // pl with the SELL arrays' row order and offset widths
  DevState* st = nullptr;
  DevState* st_host = nullptr;  // pinned, 2 slots
  hipEvent_t ev[2] = {nullptr, nullptr};
  // refinement mode
  int precision = BCG_FP64;
  double inner_tol = 0.0;  // 0: by group width (effective_inner_tol)
  int inner_maxit = 1000, max_outer = 50;
  float *R32 = nullptr, *P32 = nullptr, *Q32 = nullptr, *D32 = nullptr;
  int chunk = 32;       // upper bound on iterations enqueued per poll
  RowPath path = RowPath::generic;  // row kernels of the current solve
  // per-kernel-class event timing
  struct ProfRec {
    int cls, it;
    hipEvent_t a, b;
  };
  bool prof_on = false;
  unsigned prof_mask = 0;  // classes bracketed by events
  std::vector<hipEvent_t> ev_pool;
  std::vector<ProfRec> prof_recs;
  bcg_kernel_time prof[BCG_NUM_KERNEL_CLASSES]{};
  std::vector<double> ref_r0;  // host copy of the stop rule's reference norms
  double known_true = -1.0;    // true relative residual of the returned X, when the solve measured it
  bcg_info info{};
  std::vector<double> host_ratios;
  // Jacobi preconditioning by symmetric scaling
  int precond = BCG_PRECOND_NONE;
  double* dscale = nullptr;   // diag(A)^{-1/2}
  double* vals_s = nullptr;   // values of D^{-1/2} A D^{-1/2}
  float* vals32_s = nullptr;
  double* Bs = nullptr;       // D^{-1/2} B of the current solve
  std::vector<double> true_r0;  // ||B - A X0||_j of the current solve
};

namespace {

void free_all(bcg_handle* h) {
  void* ptrs[] = {h->rowptr, h->colind, h->vals, h->vals32, h->R, h->P, h->Q, h->partA, h->part2, h->partR, h->partN,
                  h->alpha, h->rho, h->rnew, h->lam, h->beta, h->ws, h->lam32, h->beta32, h->r0, h->ratios,
                  h->scale, h->st, h->R32, h->P32, h->Q32, h->D32, h->sched, h->dscale, h->vals_s,
                  h->vals32_s, h->Bs, h->sl_ptr, h->sl_perm, h->sl_col, h->sl_map, h->sl_val, h->sl_val32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (h->st_host) (void)hipHostFree(h->st_host);
  for (auto& e : h->ev)
    if (e) (void)hipEventDestroy(e);
  for (auto& r : h->prof_recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (auto& e : h->ev_pool) (void)hipEventDestroy(e);
}

hipEvent_t pool_event(bcg_handle* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Launches `f` (one kernel class), bracketed by events when profiling.
template <typename F>
void timed(bcg_handle* h, int cls, int it, F&& f) {
  if (!h->prof_on || !((h->prof_mask >> cls) & 1u)) {
    f();
    return;
  }
  hipEvent_t a = pool_event(h), b = pool_event(h);
  (void)hipEventRecord(a, h->stream);
  f();
  (void)hipEventRecord(b, h->stream);
  h->prof_recs.push_back({cls, it, a, b});
}

// Accumulates the recorded launches of iterations <= last_it (0 = set-up
// launches); the others returned at entry and are dropped. Stream must be idle.
void prof_collect(bcg_handle* h, int last_it) {
  for (auto& r : h->prof_recs) {
    if (r.it <= last_it) {
      float ms = 0.0f;
      if (hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
        h->prof[r.cls].launches += 1;
        h->prof[r.cls].total_ms += ms;
      }
    }
    h->ev_pool.push_back(r.a);
    h->ev_pool.push_back(r.b);
  }
  h->prof_recs.clear();
}

int alloc_fp32(bcg_handle* h) {
  if (h->R32) return BCG_OK;
  const size_t nk = static_cast<size_t>(h->n) * h->k;
  int rc;
  if ((rc = dalloc(&h->R32, nk)) || (rc = dalloc(&h->P32, nk)) || (rc = dalloc(&h->Q32, nk)) ||
      (rc = dalloc(&h->D32, nk)))
    return rc;
  return BCG_OK;
}

int reset_state(bcg_handle* h) {
  DevState z{};
  HIP_TRY(hipMemcpyAsync(h->st, &z, sizeof z, hipMemcpyHostToDevice, h->stream));
  return BCG_OK;
}

int read_state(bcg_handle* h, DevState* out) {
  if (!h->st_host) {  // a handle without pinned state slots (the allocation-free solve)
    HIP_TRY(hipMemcpyAsync(out, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return BCG_OK;
  }
  HIP_TRY(hipMemcpyAsync(h->st_host, h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  *out = h->st_host[0];
  return BCG_OK;
}

// Norms^2 of the k columns (the tail of a reduced partial row) to the host.
int fetch_norms(bcg_handle* h, const double* red, std::vector<double>& out) {
  out.resize(h->k);
  HIP_TRY(hipMemcpyAsync(out.data(), red + h->pl.E, sizeof(double) * h->k, hipMemcpyDeviceToHost, h->stream));
  HIP_TRY(hipStreamSynchronize(h->stream));
  return BCG_OK;
}

bool decoupled(const bcg_handle* h) { return h->p == 1 && (h->variant == BCG_PARALLEL || h->variant == BCG_HYBRID); }

// X += P lambda; unless `last`: P = R + P beta and the partial <<P, R>>
// (line 6 of the next iteration) in partR.
template <typename T>
void enqueue_update_xp(bcg_handle* h, const IterBuffers<T>& b, int it) {
  const Plan& pl = h->pl;
  hipStream_t s = h->stream;
  const bool mfma = h->path == RowPath::mfma, fast = mfma || h->path == RowPath::fast;
  const bool vec = mfma && (pl.upd_vec[std::is_same<T, float>::value ? 1 : 0] & 2);
  timed(h, BCG_K_UPDATE_XP, it, [&] {
    if (mfma && !vec)
      launch_update_xp_mfma<T>(pl, b.X, b.P, b.R, b.lam, b.beta, h->partR, h->st, s);
    else if (fast)
      launch_update_xp_fast<T>(pl, b.X, b.P, b.R, b.lam, b.beta, h->partR, h->st, s);
    else
      launch_update_xp<T>(pl, b.X, b.P, b.R, b.lam, b.beta, h->partR, h->st, s);
  });
  if (!fast && !pl.fused)
    timed(h, BCG_K_PRODUCT, it + 1, [&] { launch_product<T>(pl, b.P, b.R, h->partR, h->st, s); });
}

// Enqueues one iteration (number `it`) of Algorithm 1 in precision T.
template <typename T>
void enqueue_iteration(bcg_handle* h, const IterBuffers<T>& b, double tol, int it, int maxit) {
  const Plan& pl = h->pl;
  hipStream_t s = h->stream;
  const bool mfma = h->path == RowPath::mfma, fast = mfma || h->path == RowPath::fast;
  timed(h, BCG_K_SPMM, it, [&] {  // lines 4-5
    if (mfma && h->sell) {
      const T* sv;
      if constexpr (std::is_same<T, float>::value)
        sv = h->sl_val32;
      else
        sv = h->sl_val;
      launch_spmm_mfma<T>(h->pl_sell, h->sl_ptr, h->sl_col, sv, b.P, b.Q, h->partA, h->st, s);
    } else if (mfma)
      launch_spmm_mfma<T>(pl, h->rowptr, h->colind, b.vals, b.P, b.Q, h->partA, h->st, s);
    else if (fast)
      launch_spmm_fast<T>(pl, h->rowptr, h->colind, b.vals, b.P, b.Q, h->partA, h->st, s);
    else
      launch_spmm_product<T>(pl, h->rowptr, h->colind, b.vals, b.P, b.Q, h->partA, h->st, s);
  });
  if (!fast && !pl.fused) timed(h, BCG_K_PRODUCT, it, [&] { launch_product<T>(pl, b.P, b.Q, h->partA, h->st, s); });
  const int sp_rows = mfma ? pl.sp_nwg[std::is_same<T, float>::value ? 1 : 0] : pl.nwg;
  // line 6 (rho of the previous X/P pass; the set-up reduced the first) and
  // line 7
  timed(h, BCG_K_SMALL, it, [&] {
    launch_reduce_lambda(pl, h->partA, sp_rows, h->part2, h->partR, it > 1 ? pl.nwg : 0, h->alpha, h->rho, h->lam,
                         h->lam32, h->ws, h->st, s);
  });
  const bool vec = mfma && (pl.upd_vec[std::is_same<T, float>::value ? 1 : 0] & 1);
  timed(h, BCG_K_UPDATE_R, it, [&] {  // line 9 and the product of line 11
    if (mfma && !vec)
      launch_update_r_mfma<T>(pl, b.R, b.Q, b.lam, h->partN, h->st, s);
    else if (fast)
      launch_update_r_fast<T>(pl, b.R, b.Q, b.lam, h->partN, h->st, s);
    else
      launch_update_r<T>(pl, b.R, b.Q, b.lam, h->partN, h->st, s);
  });
  if (!fast && !pl.fused) timed(h, BCG_K_PRODUCT, it, [&] { launch_product<T>(pl, b.R, b.R, h->partN, h->st, s); });
  timed(h, BCG_K_SMALL, it, [&] {  // stop rule, line 12
    launch_reduce_beta(pl, h->partN, pl.nwg, h->rnew, h->r0, h->rho, h->beta, h->beta32, h->ws, h->ratios, h->st, tol,
                       it, maxit, s);
  });
  // line 8 and line 13 with the partial products of line 6 for the next
  // iteration (on the last iteration only line 8)
  enqueue_update_xp<T>(h, b, it);
}

// Iterations to enqueue next: half the predicted remaining count (from the
// observed geometric decrease of the largest ratio), at least 1, at most
// h->chunk; keeps the launches enqueued past the stop iteration few.
int next_chunk(const bcg_handle* h, double tol, int enq, int it_a, double r_a, int it_b, double r_b) {
  const int cap = h->chunk;
  if (!(tol > 0.0) || it_b <= it_a || !(r_a > 0.0) || !(r_b > 0.0) || !(r_b < r_a)) return cap;
  const double rate = (std::log(r_b) - std::log(r_a)) / (it_b - it_a);  // < 0
  const double remaining = (std::log(tol) - std::log(r_b)) / rate - (enq - it_b);
  if (!(remaining < 1e9)) return cap;
  const int c = static_cast<int>(std::ceil(0.5 * remaining));
  return std::max(1, std::min(cap, c));
}

// Runs iterations 1..maxit until the device flags completion; rho must hold
// the reduced <<P^1, R^0>> and r0 the reference norms.
template <typename T>
int run_iterations(bcg_handle* h, const IterBuffers<T>& b, double tol, int maxit, DevState* final_state) {
  int enq = 0;
  int slot_head = 0, inflight = 0;
  int it_a = 0, it_b = 0;
  double r_a = 0.0, r_b = 0.0;
  auto enqueue_chunk = [&](int slot, int want) -> int {
    const int c = std::min(want, maxit - enq);
    for (int j = 0; j < c; ++j) enqueue_iteration<T>(h, b, tol, enq + 1 + j, maxit);
    enq += c;
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(&h->st_host[slot], h->st, sizeof(DevState), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipEventRecord(h->ev[slot], h->stream));
    return BCG_OK;
  };
  const int first = std::min(h->chunk, 8);
  int rc;
  if (!h->st_host) {
    // no pinned state slots or events (the allocation-free solve): one chunk
    // at a time, its state read back synchronously
    int want = first;
    while (enq < maxit) {
      const int c = std::min(want, maxit - enq);
      for (int j = 0; j < c; ++j) enqueue_iteration<T>(h, b, tol, enq + 1 + j, maxit);
      enq += c;
      HIP_TRY(hipGetLastError());
      DevState seen{};
      if ((rc = read_state(h, &seen))) return rc;
      if (seen.done || seen.last) break;
      it_a = it_b;
      r_a = r_b;
      it_b = seen.iter;
      r_b = seen.max_ratio;
      want = next_chunk(h, tol, enq, it_a, r_a, it_b, r_b);
    }
    rc = read_state(h, final_state);
    if (h->prof_on) prof_collect(h, final_state->iter);
    return rc;
  }
  if (maxit > 0) {
    if ((rc = enqueue_chunk(0, first))) return rc;
    inflight = 1;
    if (enq < maxit) {
      if ((rc = enqueue_chunk(1, first))) return rc;
      inflight = 2;
    }
  }
  while (inflight > 0) {
    HIP_TRY(hipEventSynchronize(h->ev[slot_head]));
    const DevState seen = h->st_host[slot_head];
    --inflight;
    const int freed = slot_head;
    slot_head ^= 1;
    if (seen.done || seen.last) break;
    it_a = it_b;
    r_a = r_b;
    it_b = seen.iter;
    r_b = seen.max_ratio;
    if (enq < maxit) {
      if ((rc = enqueue_chunk(freed, next_chunk(h, tol, enq, it_a, r_a, it_b, r_b)))) return rc;
      ++inflight;
    }
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  rc = read_state(h, final_state);
  if (h->prof_on) prof_collect(h, final_state->iter);
  return rc;
}

// Sets r0 (device) from host norms^2; applies the input checks of the paper's
// reading (zero columns only in the diagonal subalgebra).
int set_reference(bcg_handle* h, const std::vector<double>& norms2, std::vector<double>& r0, bool* all_zero,
                  bool allow_zero) {
  r0.resize(h->k);
  bool any_zero = false;
  *all_zero = true;
  for (int j = 0; j < h->k; ++j) {
    const double v = std::sqrt(norms2[j]);
    if (!std::isfinite(v)) return fail(BCG_EINVAL, "non-finite initial residual in column %d", j);
    r0[j] = v;
    if (v == 0.0)
      any_zero = true;
    else
      *all_zero = false;
  }
  if (any_zero && !*all_zero && !allow_zero)
    return fail(BCG_EINVAL, "zero initial residual column with a non-diagonal subalgebra");
  HIP_TRY(hipMemcpyAsync(h->r0, r0.data(), sizeof(double) * h->k, hipMemcpyHostToDevice, h->stream));
  return BCG_OK;
}

double max_ratio(const std::vector<double>& norms2, const std::vector<double>& r0) {
  double m = 0.0;
  for (size_t j = 0; j < r0.size(); ++j) {
    const double v = r0[j] == 0.0 ? 0.0 : std::sqrt(norms2[j]) / r0[j];
    if (!std::isfinite(v)) return NAN;
    m = std::max(m, v);
  }
  return m;
}

// Plain FP64 solve from the current X. ref_r0 (host, optional) replaces the
// initial residual norms in the stop rule.
int solve_fp64(bcg_handle* h, const double* B, double* X, double tol, int maxit, const std::vector<double>* ref_r0,
               int* iterations) {
  const Plan& pl = h->pl;
  int rc;
  *iterations = 0;
  if ((rc = reset_state(h))) return rc;
  timed(h, BCG_K_RESIDUAL, 0, [&] {  // lines 1-2
    launch_residual(pl, h->rowptr, h->colind, h->vals, B, X, h->R, h->P, h->partR, 1, h->stream);
  });
  if (!pl.fused)
    timed(h, BCG_K_PRODUCT, 0, [&] { launch_product<double>(pl, h->R, h->R, h->partR, nullptr, h->stream); });
  timed(h, BCG_K_REDUCE, 0, [&] { launch_reduce(pl, h->partR, h->rho, pl.W, nullptr, h->stream); });
  HIP_TRY(hipGetLastError());
  std::vector<double> norms2, r0;
  if ((rc = fetch_norms(h, h->rho, norms2))) return rc;
  bool all_zero = false;
  if (ref_r0) {
    for (int j = 0; j < h->k; ++j)
      if (!std::isfinite(norms2[j])) return fail(BCG_EINVAL, "non-finite residual in column %d", j);
    r0 = *ref_r0;
    all_zero = true;
    for (double v : r0) all_zero &= (v == 0.0);
    HIP_TRY(hipMemcpyAsync(h->r0, r0.data(), sizeof(double) * h->k, hipMemcpyHostToDevice, h->stream));
  } else if ((rc = set_reference(h, norms2, r0, &all_zero, decoupled(h)))) {
    return rc;
  }
  h->ref_r0 = r0;
  for (int j = 0; j < h->k; ++j) h->host_ratios[j] = r0[j] == 0.0 ? 0.0 : std::sqrt(norms2[j]) / r0[j];
  if (all_zero) return BCG_OK;
  if (maxit == 0) return BCG_NOT_CONVERGED;
  IterBuffers<double> b{h->vals, X, h->R, h->P, h->Q, h->lam, h->beta};
  h->path = row_path(h->pl, reinterpret_cast<uintptr_t>(X) % 16 == 0);
  DevState fin{};
  if ((rc = run_iterations<double>(h, b, tol, maxit, &fin))) return rc;
  *iterations = fin.iter;
  if (fin.iter > 0)
    HIP_TRY(hipMemcpy(h->host_ratios.data(), h->ratios, sizeof(double) * h->k, hipMemcpyDeviceToHost));
  if (!fin.done && !fin.last) return BCG_NOT_CONVERGED;
  return fin.status;
}

// Reduction asked of the next inner FP32 solve: the remaining factor
// 0.5 tol / ratio, but no deeper than inner_tol / 4 (a deep first solve saves
// the restart of a second one where FP32 delivers the depth).
double inner_target(double inner_tol, double tol, double ratio) {
  const double need = 0.5 * tol / ratio;
  if (!(need > 0.0) || need >= 1.0) return inner_tol;
  return std::min(std::max(need, 0.25 * inner_tol), 0.5);
}

// inner_tol 0: 4e-6 for groups of p <= 16, 1e-4 for wider groups
double effective_inner_tol(double inner_tol, int p) { return inner_tol > 0.0 ? inner_tol : (p <= 16 ? 4e-6 : 1e-4); }

// Mixed precision: FP32 inner block CG, FP64 outer iterative refinement.
int solve_refine(bcg_handle* h, const double* B, double* X, double tol, int maxit) {
  const Plan& pl = h->pl;
  int rc;
  if ((rc = alloc_fp32(h))) return rc;
  bcg_info& info = h->info;
  // true FP64 residual and its column norms
  timed(h, BCG_K_RESIDUAL, 0, [&] {
    launch_residual(pl, h->rowptr, h->colind, h->vals, B, X, h->R, nullptr, h->partN, 0, h->stream);
  });
  timed(h, BCG_K_REDUCE, 0, [&] { launch_reduce(pl, h->partN, h->rnew, pl.W, nullptr, h->stream); });
  HIP_TRY(hipGetLastError());
  std::vector<double> norms2, r0;
  if ((rc = fetch_norms(h, h->rnew, norms2))) return rc;
  bool all_zero = false;
  if ((rc = set_reference(h, norms2, r0, &all_zero, decoupled(h)))) return rc;
  h->ref_r0 = r0;
  if (all_zero) return BCG_OK;
  double prev = INFINITY;
  for (int outer = 1;; ++outer) {
    const double ratio = max_ratio(norms2, r0);
    for (int j = 0; j < h->k; ++j) h->host_ratios[j] = r0[j] == 0.0 ? 0.0 : std::sqrt(norms2[j]) / r0[j];
    if (!(ratio == ratio)) return fail(BCG_EBREAKDOWN, "non-finite residual during refinement");
    if (ratio <= tol) return BCG_OK;
    bool fallback = ratio > 0.5 * prev;
    if (!fallback && outer > h->max_outer) return BCG_NOT_CONVERGED;
    if (!fallback) {
      prev = ratio;
      // inner FP32 solve of A D = R / s from D = 0
      if ((rc = reset_state(h))) return rc;
      timed(h, BCG_K_RESIDUAL, 0, [&] {
        launch_cast_init(pl, h->R, h->rnew + pl.E, h->R32, h->P32, h->D32, h->scale, h->partR, h->stream);
      });
      if (!pl.fused)
        timed(h, BCG_K_PRODUCT, 0, [&] { launch_product<float>(pl, h->R32, h->R32, h->partR, nullptr, h->stream); });
      timed(h, BCG_K_REDUCE, 0, [&] { launch_reduce(pl, h->partR, h->rho, pl.W, nullptr, h->stream); });
      std::vector<double> in2, rin;
      if ((rc = fetch_norms(h, h->rho, in2))) return rc;
      bool inner_zero = false;
      rc = set_reference(h, in2, rin, &inner_zero, decoupled(h));
      if (rc == BCG_EINVAL) {
        fallback = true;
      } else if (rc) {
        return rc;
      } else {
        IterBuffers<float> b{h->vals32, h->D32, h->R32, h->P32, h->Q32, h->lam32, h->beta32};
        h->path = row_path(h->pl, true);
        DevState fin{};
        const double itol = inner_target(effective_inner_tol(h->inner_tol, h->p), tol, ratio);
        if ((rc = run_iterations<float>(h, b, itol, h->inner_maxit, &fin)))
          return rc;
        info.iterations += fin.iter;
        info.outer_iterations = outer;
        if (fin.status < 0) {
          fallback = true;
        } else {
          timed(h, BCG_K_RESIDUAL, 0, [&] { launch_axpy_scaled(h->n * h->k, X, h->D32, h->scale, h->stream); });
          timed(h, BCG_K_RESIDUAL, 0, [&] {
            launch_residual(pl, h->rowptr, h->colind, h->vals, B, X, h->R, nullptr, h->partN, 0, h->stream);
          });
          timed(h, BCG_K_REDUCE, 0, [&] { launch_reduce(pl, h->partN, h->rnew, pl.W, nullptr, h->stream); });
          HIP_TRY(hipGetLastError());
          if ((rc = fetch_norms(h, h->rnew, norms2))) return rc;
          continue;
        }
      }
    }
    // stagnation or inner breakdown: finish with the FP64 iteration from X
    info.fp64_fallback = 1;
    int its = 0;
    rc = solve_fp64(h, B, X, tol, maxit, &r0, &its);
    info.iterations += its;
    return rc;
  }
}

// Default replacement threshold of the residual-replacement form: 1e-2 for
// groups of p <= 16, 1e-1 for wider ones, whose FP32 block iterates lose
// accuracy sooner (measured: 512^2 diffusion, block 32: 765 FP32 iterations
// with 8 corrections at 0.1, 811 with 4 at 0.01; 256^3 Poisson, hybrid 16:
// 574 either way, 4 corrections fewer at 0.01).
double effective_delta(double inner_tol, int p) { return inner_tol > 0.0 ? inner_tol : (p <= 16 ? 1e-2 : 1e-1); }

// Mixed precision with residual replacement: one FP32 iteration of
// Algorithm 1 on the scaled system A D = R / s whose search direction is kept
// across the FP64 corrections. It runs until its recursive residual (in units
// of the true relative residual) reaches max(tol, delta * last), where last is
// the true relative residual at the previous correction; then X += s D, the
// FP64 residual R = B - A X replaces the FP32 one in a new scale s', P32 and
// the last line-6 product rho are rescaled by s / s' and (s / s')^2, and the
// iteration resumes at line 10 (rho_new, beta, P = R + P beta; the X/P pass
// runs with lambda = 0, so D stays 0).
int solve_reliable(bcg_handle* h, const double* B, double* X, double tol, int maxit) {
  const Plan& pl = h->pl;
  int rc;
  if ((rc = alloc_fp32(h))) return rc;
  bcg_info& info = h->info;
  const double delta = effective_delta(h->inner_tol, h->p);
  timed(h, BCG_K_RESIDUAL, 0, [&] {
    launch_residual(pl, h->rowptr, h->colind, h->vals, B, X, h->R, nullptr, h->partN, 0, h->stream);
  });
  timed(h, BCG_K_REDUCE, 0, [&] { launch_reduce(pl, h->partN, h->rnew, pl.W, nullptr, h->stream); });
  HIP_TRY(hipGetLastError());
  std::vector<double> norms2, r0;
  if ((rc = fetch_norms(h, h->rnew, norms2))) return rc;
  bool all_zero = false;
  if ((rc = set_reference(h, norms2, r0, &all_zero, decoupled(h)))) return rc;
  h->ref_r0 = r0;
  if (all_zero) return BCG_OK;
  auto scale_of = [&](const std::vector<double>& n2) {
    double m = 0.0;
    for (double v : n2) m = std::max(m, std::sqrt(v));
    return m;
  };
  IterBuffers<float> b{h->vals32, h->D32, h->R32, h->P32, h->Q32, h->lam32, h->beta32};
  h->path = row_path(h->pl, true);
  // fresh start: R32 = R / s, P32 = R32, D32 = 0, rho = <<R32, R32>>
  double s = scale_of(norms2);
  if ((rc = reset_state(h))) return rc;
  timed(h, BCG_K_RESIDUAL, 0, [&] {
    launch_cast_init(pl, h->R, h->rnew + pl.E, h->R32, h->P32, h->D32, h->scale, h->partR, h->stream);
  });
  if (!pl.fused)
    timed(h, BCG_K_PRODUCT, 0, [&] { launch_product<float>(pl, h->R32, h->R32, h->partR, nullptr, h->stream); });
  timed(h, BCG_K_REDUCE, 0, [&] { launch_reduce(pl, h->partR, h->rho, pl.W, nullptr, h->stream); });
  // stop rule of the FP32 iteration in units of the true relative residual
  std::vector<double> ref(h->k);
  auto set_ref = [&](double sc) -> int {
    for (int j = 0; j < h->k; ++j) ref[j] = r0[j] / sc;
    HIP_TRY(hipMemcpyAsync(h->r0, ref.data(), sizeof(double) * h->k, hipMemcpyHostToDevice, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));  // ref is reused
    return BCG_OK;
  };
  if ((rc = set_ref(s))) return rc;
  double last = max_ratio(norms2, r0);
  bool fallback = false;
  int corrections = 0;
  for (;;) {
    const double itol = std::max(tol, delta * last);
    DevState fin{};
    if ((rc = run_iterations<float>(h, b, itol, h->inner_maxit, &fin))) return rc;
    info.iterations += fin.iter;
    if (fin.status < 0) {
      fallback = true;  // FP32 breakdown: the FP64 iteration from the last correction's X
      break;
    }
    // correction and true residual
    timed(h, BCG_K_RESIDUAL, 0, [&] { launch_axpy_scaled(h->n * h->k, X, h->D32, h->scale, h->stream); });
    timed(h, BCG_K_RESIDUAL, 0, [&] {
      launch_residual(pl, h->rowptr, h->colind, h->vals, B, X, h->R, nullptr, h->partN, 0, h->stream);
    });
    timed(h, BCG_K_REDUCE, 0, [&] { launch_reduce(pl, h->partN, h->rnew, pl.W, nullptr, h->stream); });
    HIP_TRY(hipGetLastError());
    if ((rc = fetch_norms(h, h->rnew, norms2))) return rc;
    ++corrections;
    info.outer_iterations = corrections;
    const double ratio = max_ratio(norms2, r0);
    for (int j = 0; j < h->k; ++j) h->host_ratios[j] = r0[j] == 0.0 ? 0.0 : std::sqrt(norms2[j]) / r0[j];
    if (!(ratio == ratio)) return fail(BCG_EBREAKDOWN, "non-finite residual during refinement");
    if (ratio <= tol) {
      h->known_true = ratio;  // the residual of the X the solve returns
      return BCG_OK;
    }
    if (!(ratio <= 0.5 * last)) {
      fallback = true;  // no progress since the last correction
      break;
    }
    if (corrections >= h->max_outer) {
      h->known_true = ratio;
      return BCG_NOT_CONVERGED;
    }
    last = ratio;
    // residual replacement in the new scale s'
    const double s_new = scale_of(norms2), f = s / s_new;
    s = s_new;
    if ((rc = set_ref(s))) return rc;
    if ((rc = reset_state(h))) return rc;
    timed(h, BCG_K_SMALL, 0, [&] { launch_scale_vec(h->rho, pl.E, f * f, h->stream); });
    timed(h, BCG_K_RESIDUAL, 0, [&] {
      launch_cast_init(pl, h->R, h->rnew + pl.E, h->R32, h->P32, h->D32, h->scale, h->partN, h->stream, f);
    });
    if (!pl.fused)
      timed(h, BCG_K_PRODUCT, 0, [&] { launch_product<float>(pl, h->R32, h->R32, h->partN, nullptr, h->stream); });
    // line 10-12 with the replaced residual (no stop: its ratio is above itol)
    timed(h, BCG_K_SMALL, 0, [&] {
      launch_reduce_beta(pl, h->partN, pl.nwg, h->rnew, h->r0, h->rho, h->beta, h->beta32, h->ws, h->ratios, h->st,
                         std::max(tol, delta * last), 0, INT32_MAX, h->stream);
    });
    // line 13 (lambda = 0 leaves D = 0) and the next iteration's line 6
    HIP_TRY(hipMemsetAsync(h->lam32, 0, sizeof(float) * pl.E, h->stream));
    enqueue_update_xp<float>(h, b, 0);
    timed(h, BCG_K_REDUCE, 0, [&] { launch_reduce(pl, h->partR, h->rho, pl.W, nullptr, h->stream); });
    HIP_TRY(hipGetLastError());
    DevState chk{};
    if ((rc = read_state(h, &chk))) return rc;
    if (chk.done || chk.last) {
      if (chk.status < 0) {
        fallback = true;  // beta breakdown after the replacement
        break;
      }
      return fail(BCG_EHIP, "residual replacement: the stop rule fired on the replaced residual");
    }
  }
  (void)fallback;
  info.fp64_fallback = 1;
  int its = 0;
  rc = solve_fp64(h, B, X, tol, maxit, &r0, &its);
  info.iterations += its;
  return rc;
}

void free_sell(bcg_handle* h) {
  void* ptrs[] = {h->sl_ptr, h->sl_perm, h->sl_col, h->sl_map, h->sl_val, h->sl_val32};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  h->sl_ptr = h->sl_perm = h->sl_col = h->sl_map = nullptr;
  h->sl_val = nullptr;
  h->sl_val32 = nullptr;
  h->sell_slots = 0;
}

// SELL-16-sigma layout of a CSR pattern, built on the host. Positions
// follow `order_in` (natural order when NULL); within each window of sigma
// positions the rows are sorted by decreasing length (stable). Slice S
// holds positions 16 S .. 16 S + 15 (positions past n repeat the last row and
// are masked by the kernels) and is as wide as its longest row (at least 1).
// Its two halves of 8 positions follow each other, slot by slot: slot t of
// position 8 h + r of slice S is entry ptr[S] + 8 w h + 8 t + r, the row's
// t-th CSR entry, or padding (column = the row, map = -1, value 0).
int sell_layout_host(int64_t n, const int32_t* rp, const int32_t* ci, const int32_t* order_in, int sigma,
                     std::vector<int32_t>& sp, std::vector<int32_t>& perm, std::vector<int32_t>& col,
                     std::vector<int32_t>& map) {
  std::vector<int32_t> order(n);
  for (int64_t i = 0; i < n; ++i) order[i] = order_in ? order_in[i] : static_cast<int32_t>(i);
  auto len = [&](int32_t r) { return rp[r + 1] - rp[r]; };
  if (sigma > 1)
    for (int64_t w0 = 0; w0 < n; w0 += sigma)
      std::stable_sort(order.begin() + w0, order.begin() + std::min<int64_t>(n, w0 + sigma),
                       [&](int32_t a, int32_t b) { return len(a) > len(b); });
  const int64_t ns = (n + 15) / 16;
  sp.assign(ns + 1, 0);
  perm.assign(ns * 16, 0);
  std::vector<int32_t> width(ns);
  int64_t slots = 0;
  for (int64_t S = 0; S < ns; ++S) {
    int w = 1;
    for (int r = 0; r < 16; ++r) {
      const int64_t pos = 16 * S + r;
      perm[pos] = order[pos < n ? pos : n - 1];
      if (pos < n) w = std::max(w, len(perm[pos]));
    }
    width[S] = w;
    sp[S] = static_cast<int32_t>(slots);
    slots += 16 * static_cast<int64_t>(w);
    if (slots > INT32_MAX) return fail(BCG_EINVAL, "SELL storage needs more than 2^31 - 1 slots");
  }
  sp[ns] = static_cast<int32_t>(slots);
  col.assign(slots, 0);
  map.assign(slots, 0);
  for (int64_t S = 0; S < ns; ++S)
    for (int r = 0; r < 16; ++r) {
      const int64_t pos = 16 * S + r;
      const int32_t row = perm[pos];
      const int l = pos < n ? len(row) : 0;
      for (int t = 0; t < width[S]; ++t) {
        const int64_t e = sp[S] + 8 * static_cast<int64_t>(width[S]) * (r >> 3) + 8 * t + (r & 7);
        col[e] = t < l ? ci[rp[row] + t] : row;
        map[e] = t < l ? rp[row] + t : -1;
      }
    }
  return BCG_OK;
}

// The handle's SELL copy: the layout of its pattern in its row schedule,
// uploaded, and the plan of the sparse product on it.
int build_sell(bcg_handle* h) {
  const int64_t n = h->n, nnz = h->nnz;
  std::vector<int32_t> rp(n + 1), ci(nnz > 0 ? nnz : 1), order;
  HIP_TRY(hipMemcpy(rp.data(), h->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  if (nnz > 0) HIP_TRY(hipMemcpy(ci.data(), h->colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  if (h->pl.sched) {
    order.resize(n);
    HIP_TRY(hipMemcpy(order.data(), h->pl.sched, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
  }
  std::vector<int32_t> sp, perm, col, map;
  int rc = sell_layout_host(n, rp.data(), ci.data(), h->pl.sched ? order.data() : nullptr, h->sell_sigma, sp, perm,
                            col, map);
  if (rc) return rc;
  const int64_t ns = (n + 15) / 16, slots = sp[ns];
  if ((rc = dalloc(&h->sl_ptr, ns + 1)) || (rc = dalloc(&h->sl_perm, ns * 16)) || (rc = dalloc(&h->sl_col, slots)) ||
      (rc = dalloc(&h->sl_map, slots)) || (rc = dalloc(&h->sl_val, slots)) || (rc = dalloc(&h->sl_val32, slots)))
    return rc;
  HIP_TRY(hipMemcpy(h->sl_ptr, sp.data(), sizeof(int32_t) * (ns + 1), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->sl_perm, perm.data(), sizeof(int32_t) * ns * 16, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->sl_col, col.data(), sizeof(int32_t) * slots, hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(h->sl_map, map.data(), sizeof(int32_t) * slots, hipMemcpyHostToDevice));
  h->sell_slots = slots;
  Plan& ps = h->pl_sell;
  ps = h->pl;
  ps.sched = h->sl_perm;
  ps.sell = 1;
  // 32-bit byte offsets when the vectors, the slots and the slice table all
  // stay below 4 GiB (BCG_WIDE_OFFSETS forces 64-bit offsets)
  const int64_t lim = int64_t(1) << 32;
  const char* wide = std::getenv("BCG_WIDE_OFFSETS");
  const bool force_wide = wide != nullptr && wide[0] != '\0' && wide[0] != '0';
  for (int prec = 0; prec < 2; ++prec) {
    const int64_t elem = prec ? 4 : 8;
    ps.sp_o32[prec] = n * h->k * elem < lim && slots * elem < lim && ns * 16 * 4 < lim && !force_wide;
  }
  return BCG_OK;
}

// after a change of the row schedule: the SELL copy follows it
int rebuild_sell(bcg_handle* h) {
  if (!h->sell) return BCG_OK;
  h->sell = 0;
  free_sell(h);
  const int rc = build_sell(h);
  if (rc) {
    free_sell(h);
    return rc;
  }
  h->sell = 1;
  return BCG_OK;
}

// Scale factors and scaled values of the Jacobi preconditioner for the
// handle's current values. Synchronous (reads the flag).
int jacobi_prepare(bcg_handle* h) {
  int rc;
  const int64_t nz = h->nnz > 0 ? h->nnz : 1;
  if ((!h->dscale && (rc = dalloc(&h->dscale, h->n))) || (!h->vals_s && (rc = dalloc(&h->vals_s, nz))) ||
      (!h->vals32_s && (rc = dalloc(&h->vals32_s, nz))))
    return rc;
  DevState z{};
  HIP_TRY(hipMemcpyAsync(h->st, &z, sizeof z, hipMemcpyHostToDevice, h->stream));
  launch_jacobi_scale(h->n, h->rowptr, h->colind, h->vals, h->dscale, &h->st->status, h->stream);
  HIP_TRY(hipGetLastError());
  DevState out{};
  if ((rc = read_state(h, &out))) return rc;
  if (out.status != 0) return fail(BCG_EINVAL, "Jacobi preconditioner needs a positive finite diagonal entry in every row");
  launch_scale_values(h->n, h->rowptr, h->colind, h->vals, h->dscale, h->vals_s, h->vals32_s, h->stream);
  HIP_TRY(hipGetLastError());
  return BCG_OK;
}

int validate_p(int variant, int k, int p, int* p_out) {
  if (k < 1 || k > 256) return fail(BCG_EINVAL, "k=%d outside 1..256", k);
  switch (variant) {
    case BCG_BLOCK:
      if (p != 0 && p != k) return fail(BCG_EINVAL, "block subalgebra needs p = k or 0 (got %d)", p);
      *p_out = k;
      return BCG_OK;
    case BCG_PARALLEL:
      if (p != 0 && p != 1) return fail(BCG_EINVAL, "parallel subalgebra needs p = 1 or 0 (got %d)", p);
      *p_out = 1;
      return BCG_OK;
    case BCG_GLOBAL:
      if (p == 0) {
        *p_out = 1;
        return BCG_OK;
      }
      [[fallthrough]];
    case BCG_HYBRID:
      if (p < 1 || p > k || k % p) return fail(BCG_EINVAL, "p=%d must divide k=%d", p, k);
      *p_out = p;
      return BCG_OK;
    default:
      return fail(BCG_EINVAL, "unknown subalgebra %d", variant);
  }
}

}  // namespace

// Workspace of bcg_solve_noalloc: one array per GPU the library runs on,
// held until the process ends. Host code never uses its name as an address:
// each device's copy is reached through the pointer hipGetSymbolAddress
// returns for that device.
constexpr size_t kScratchBytes = size_t(128) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxDevices] = {};

// Address of the current device's scratch array (looked up once per device).
int scratch_address(int device, unsigned char** out) {
  if (device < 0 || device >= kMaxDevices) return fail(BCG_EINVAL, "device %d outside 0..%d", device, kMaxDevices - 1);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(BCG_EHIP, "hipGetSymbolAddress(scratch) failed on device %d: %s", device, hipGetErrorString(e));
    g_scratch_ptr[device] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[device];
  return BCG_OK;
}

// Consecutive 256-byte aligned slices of the scratch array (base nullptr:
// only the total is counted).
struct Carve {
  unsigned char* base;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~size_t(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += (count ? count : 1) * sizeof(T);
    return p;
  }
};

// Points every workspace buffer of an FP64 solve into `c` (as bcg_create
// sizes them; the matrix stays the caller's).
void carve_workspace(bcg_handle& h, Carve& c) {
  const Plan& pl = h.pl;
  const size_t nk = static_cast<size_t>(h.n) * h.k;
  h.R = c.take<double>(nk);
  h.P = c.take<double>(nk);
  h.Q = c.take<double>(nk);
  h.partA = c.take<double>(static_cast<size_t>(std::max({pl.nwg, pl.sp_nwg[0], pl.sp_nwg[1]})) * pl.W);
  h.part2 = c.take<double>(static_cast<size_t>(kRedSplits) * pl.W);
  h.partR = c.take<double>(static_cast<size_t>(pl.nwg) * pl.W);
  h.partN = c.take<double>(static_cast<size_t>(pl.nwg) * pl.W);
  h.alpha = c.take<double>(pl.W);
  h.rho = c.take<double>(pl.W);
  h.rnew = c.take<double>(pl.W);
  h.lam = c.take<double>(pl.E);
  h.beta = c.take<double>(pl.E);
  h.lam32 = c.take<float>(pl.E);
  h.beta32 = c.take<float>(pl.E);
  h.ws = c.take<double>(pl.p > 48 ? static_cast<size_t>(pl.qo) * 2 * pl.p * pl.p : 1);
  h.r0 = c.take<double>(h.k);
  h.ratios = c.take<double>(h.k);
  h.scale = c.take<double>(1);
  h.st = c.take<DevState>(1);
}

}  // namespace

extern "C" {

const char* bcg_last_error(void) { return g_error.c_str(); }

int bcg_solve_noalloc(const bcg_csr* A, int k, int subalgebra, int p, const double* B, double* X, double tol,
                      int maxit, void* hip_stream, bcg_info* info) {
  g_error.clear();
  if (!A || !A->rowptr || !A->colind || !A->values) return fail(BCG_EINVAL, "CSR arrays must be non-NULL");
  if (A->n < 1 || A->n >= INT32_MAX || A->nnz < 0 || A->nnz >= INT32_MAX)
    return fail(BCG_EINVAL, "n=%lld nnz=%lld outside the int32 index range", (long long)A->n, (long long)A->nnz);
  if (!B || !X || static_cast<const void*>(B) == static_cast<const void*>(X))
    return fail(BCG_EINVAL, "B and X must be distinct non-NULL device arrays");
  if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0) return fail(BCG_EINVAL, "tol must be finite >= 0, maxit >= 0");
  int pn = 0;
  int rc = validate_p(subalgebra, k, p, &pn);
  if (rc) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  bcg_handle h;
  h.n = A->n;
  h.nnz = A->nnz;
  h.k = k;
  h.p = pn;
  h.variant = subalgebra;
  const int dec = pn == 1 && (subalgebra == BCG_PARALLEL || subalgebra == BCG_HYBRID);
  h.pl = make_plan(h.n, h.nnz, k, pn, subalgebra == BCG_GLOBAL ? 1 : 0, dec);
  Carve need{nullptr};
  carve_workspace(h, need);
  if (need.off > kScratchBytes)
    return fail(BCG_EINVAL, "the solve needs %zu bytes of workspace; bcg_solve_noalloc holds %zu (use bcg_create)",
                need.off, kScratchBytes);
  HIP_TRY(hipGetDevice(&h.device));
  unsigned char* base = nullptr;
  if ((rc = scratch_address(h.device, &base))) return rc;
  Carve c{base};
  carve_workspace(h, c);
  h.stream = static_cast<hipStream_t>(hip_stream);
  // the caller's matrix is read in place (the kernels never write it)
  h.rowptr = const_cast<int32_t*>(A->rowptr);
  h.colind = const_cast<int32_t*>(A->colind);
  h.vals = const_cast<double*>(A->values);
  h.host_ratios.assign(k, 1.0);
  // the CSR contents, before any kernel follows a row range
  if ((rc = reset_state(&h))) return rc;
  launch_check_csr(h.rowptr, h.colind, h.n, h.nnz, &h.st->status, h.stream);
  HIP_TRY(hipGetLastError());
  DevState chk{};
  if ((rc = read_state(&h, &chk))) return rc;
  if (chk.status != 0)
    return fail(BCG_EINVAL, "malformed CSR: needs rowptr[0] = 0, rowptr non-decreasing, rowptr[n] = nnz "
                            "and every column index in [0, n)");
  h.info = bcg_info{};
  h.info.k = k;
  int its = 0;
  rc = solve_fp64(&h, B, X, tol, maxit, nullptr, &its);
  h.info.iterations = its;
  const hipError_t se = hipStreamSynchronize(h.stream);
  if (se != hipSuccess && rc >= 0) rc = fail(BCG_EHIP, "solve failed: %s", hipGetErrorString(se));
  if (rc != BCG_EINVAL && rc != BCG_EHIP && (int)h.ref_r0.size() == k) {
    launch_residual(h.pl, h.rowptr, h.colind, h.vals, B, X, h.Q, nullptr, h.partN, 0, h.stream);
    launch_reduce(h.pl, h.partN, h.rnew, h.pl.W, nullptr, h.stream);
    std::vector<double> n2;
    if (fetch_norms(&h, h.rnew, n2) == BCG_OK) h.info.true_rel_res = max_ratio(n2, h.ref_r0);
  }
  double m = 0.0;
  for (double v : h.host_ratios) m = std::max(m, v);
  h.info.max_rel_res = m;
  h.info.status = rc;
  h.info.converged = rc == BCG_OK;
  h.info.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = h.info;
  return rc;
}

int bcg_create(const bcg_csr* A, int k, int subalgebra, int p, bcg_handle** out) {
  g_error.clear();
  if (!out) return fail(BCG_EINVAL, "out is NULL");
  *out = nullptr;
  if (!A || !A->rowptr || !A->colind || !A->values) return fail(BCG_EINVAL, "CSR arrays must be non-NULL");
  if (A->n < 1 || A->n >= INT32_MAX || A->nnz < 0 || A->nnz >= INT32_MAX)
    return fail(BCG_EINVAL, "n=%lld nnz=%lld outside the int32 index range", (long long)A->n, (long long)A->nnz);
  int pn = 0;
  int rc = validate_p(subalgebra, k, p, &pn);
  if (rc) return rc;
  int device = 0;
  HIP_TRY(hipGetDevice(&device));
  auto* h = new bcg_handle();
  h->device = device;
  h->n = A->n;
  h->nnz = A->nnz;
  h->k = k;
  h->p = pn;
  h->variant = subalgebra;
  const int dec = pn == 1 && (subalgebra == BCG_PARALLEL || subalgebra == BCG_HYBRID);
  h->pl = make_plan(h->n, h->nnz, k, pn, subalgebra == BCG_GLOBAL ? 1 : 0, dec);
  if (const char* env = std::getenv("BCG_POLL_EVERY")) h->chunk = std::max(1, std::atoi(env));
  h->host_ratios.assign(k, 1.0);
  const Plan& pl = h->pl;
  const size_t nk = static_cast<size_t>(h->n) * k;
  const size_t partsz = static_cast<size_t>(pl.nwg) * pl.W;
  const size_t partasz = static_cast<size_t>(std::max({pl.nwg, pl.sp_nwg[0], pl.sp_nwg[1]})) * pl.W;
  const size_t wssz = (pl.p > 48) ? static_cast<size_t>(pl.qo) * 2 * pl.p * pl.p : 1;
  if ((rc = dalloc(&h->rowptr, h->n + 1)) || (rc = dalloc(&h->colind, h->nnz)) || (rc = dalloc(&h->vals, h->nnz)) ||
      (rc = dalloc(&h->vals32, h->nnz)) || (rc = dalloc(&h->R, nk)) || (rc = dalloc(&h->P, nk)) ||
      (rc = dalloc(&h->Q, nk)) || (rc = dalloc(&h->partA, partasz)) ||
      (rc = dalloc(&h->part2, static_cast<size_t>(kRedSplits) * pl.W)) || (rc = dalloc(&h->partR, partsz)) ||
      (rc = dalloc(&h->partN, partsz)) || (rc = dalloc(&h->alpha, pl.W)) || (rc = dalloc(&h->rho, pl.W)) ||
      (rc = dalloc(&h->rnew, pl.W)) || (rc = dalloc(&h->lam, pl.E)) || (rc = dalloc(&h->beta, pl.E)) ||
      (rc = dalloc(&h->lam32, pl.E)) || (rc = dalloc(&h->beta32, pl.E)) || (rc = dalloc(&h->ws, wssz)) ||
      (rc = dalloc(&h->r0, k)) || (rc = dalloc(&h->ratios, k)) || (rc = dalloc(&h->scale, 1)) ||
      (rc = dalloc(&h->st, 1))) {
    free_all(h);
    delete h;
    return rc;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&h->st_host), 2 * sizeof(DevState), hipHostMallocDefault) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev[0], hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&h->ev[1], hipEventDisableTiming) != hipSuccess) {
    free_all(h);
    delete h;
    return fail(BCG_EHIP, "pinned state or event allocation failed");
  }
  hipError_t e = hipMemcpy(h->rowptr, A->rowptr, sizeof(int32_t) * (h->n + 1), hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->colind, A->colind, sizeof(int32_t) * h->nnz, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) e = hipMemcpy(h->vals, A->values, sizeof(double) * h->nnz, hipMemcpyDeviceToDevice);
  if (e == hipSuccess) {
    launch_cast_values(h->nnz, h->vals, h->vals32, nullptr);
    e = hipDeviceSynchronize();
  }
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(BCG_EHIP, "copying the CSR matrix failed: %s", hipGetErrorString(e));
  }
  // the CSR contents, before any kernel follows a row range or gathers a column
  DevState z{};
  e = hipMemcpy(h->st, &z, sizeof z, hipMemcpyHostToDevice);
  if (e == hipSuccess) {
    launch_check_csr(h->rowptr, h->colind, h->n, h->nnz, &h->st->status, nullptr);
    e = hipMemcpy(&z, h->st, sizeof z, hipMemcpyDeviceToHost);
  }
  if (e != hipSuccess) {
    free_all(h);
    delete h;
    return fail(BCG_EHIP, "checking the CSR matrix failed: %s", hipGetErrorString(e));
  }
  if (z.status != 0) {
    free_all(h);
    delete h;
    return fail(BCG_EINVAL, "malformed CSR: needs rowptr[0] = 0, rowptr non-decreasing, rowptr[n] = nnz "
                            "and every column index in [0, n)");
  }
  *out = h;
  return BCG_OK;
}

void bcg_destroy(bcg_handle* h) {
  if (!h) return;
  DeviceGuard g(h->device);
  (void)hipStreamSynchronize(h->stream);
  free_all(h);
  delete h;
}

int bcg_set_stream(bcg_handle* h, void* hip_stream) {
  if (!h) return fail(BCG_EINVAL, "handle is NULL");
  h->stream = static_cast<hipStream_t>(hip_stream);
  return BCG_OK;
}

int bcg_set_precision(bcg_handle* h, int mode, double inner_tol, int inner_maxit, int max_outer) {
  if (!h) return fail(BCG_EINVAL, "handle is NULL");
  if (mode != BCG_FP64 && mode != BCG_FP32_REFINE && mode != BCG_FP32_RELIABLE)
    return fail(BCG_EINVAL, "unknown precision mode %d", mode);
  if (!(inner_tol >= 0.0 && inner_tol < 1.0)) return fail(BCG_EINVAL, "inner_tol must be in [0, 1)");
  if (inner_maxit < 1 || max_outer < 1) return fail(BCG_EINVAL, "inner_maxit and max_outer must be >= 1");
  h->precision = mode;
  h->inner_tol = inner_tol;
  h->inner_maxit = inner_maxit;
  h->max_outer = max_outer;
  return BCG_OK;
}

int bcg_solve(bcg_handle* h, const double* B, double* X, double tol, int maxit) {
  g_error.clear();
  if (!h) return fail(BCG_EINVAL, "handle is NULL");
  if (!B || !X || static_cast<const void*>(B) == static_cast<const void*>(X))
    return fail(BCG_EINVAL, "B and X must be distinct non-NULL device arrays");
  if (!(tol >= 0.0) || !std::isfinite(tol) || maxit < 0) return fail(BCG_EINVAL, "tol must be finite >= 0, maxit >= 0");
  DeviceGuard g(h->device);
  const auto t0 = std::chrono::steady_clock::now();
  h->info = bcg_info{};
  h->info.k = h->k;
  h->ref_r0.clear();
  h->known_true = -1.0;
  h->host_ratios.assign(h->k, 1.0);
  int its = 0;
  const double* Bsolve = B;
  const bool jac = h->precond == BCG_PRECOND_JACOBI;
  h->true_r0.clear();
  if (jac) {
    // ||B - A X0||_j for info.true_rel_res, then the scaled system:
    // B <- D^{-1/2} B (a copy), X <- D^{1/2} X (in place), A <- D^{-1/2} A D^{-1/2}
    int rc0;
    if (!h->Bs && (rc0 = dalloc(&h->Bs, static_cast<size_t>(h->n) * h->k))) return rc0;
    launch_residual(h->pl, h->rowptr, h->colind, h->vals, B, X, h->Q, nullptr, h->partN, 0, h->stream);
    launch_reduce(h->pl, h->partN, h->rnew, h->pl.W, nullptr, h->stream);
    HIP_TRY(hipGetLastError());
    std::vector<double> n2;
    if ((rc0 = fetch_norms(h, h->rnew, n2))) return rc0;
    for (double v : n2) h->true_r0.push_back(std::sqrt(v));
    launch_scale_rows(h->n, h->k, B, h->dscale, h->Bs, 0, h->stream);
    launch_scale_rows(h->n, h->k, X, h->dscale, X, 1, h->stream);
    std::swap(h->vals, h->vals_s);
    std::swap(h->vals32, h->vals32_s);
    Bsolve = h->Bs;
  }
  if (h->sell)
    launch_sell_values(h->sell_slots, h->sl_map, h->vals, h->vals32, h->sl_val, h->sl_val32, h->stream);
  int rc = h->precision == BCG_FP32_REFINE     ? solve_refine(h, Bsolve, X, tol, maxit)
           : h->precision == BCG_FP32_RELIABLE ? solve_reliable(h, Bsolve, X, tol, maxit)
                                               : solve_fp64(h, Bsolve, X, tol, maxit, nullptr, &its);
  if (jac) {
    std::swap(h->vals, h->vals_s);
    std::swap(h->vals32, h->vals32_s);
    launch_scale_rows(h->n, h->k, X, h->dscale, X, 0, h->stream);  // X = D^{-1/2} Y
  }
  const bool mixed = h->precision == BCG_FP32_REFINE || h->precision == BCG_FP32_RELIABLE;
  if (!mixed) h->info.iterations = its;
  const hipError_t se = hipStreamSynchronize(h->stream);
  if (se != hipSuccess && rc >= 0) rc = fail(BCG_EHIP, "solve failed: %s", hipGetErrorString(se));
  if (h->prof_on) prof_collect(h, 0);  // set-up launches still pending
  // true residual of the returned X relative to ||R0_j|| (Euclidean); the
  // residual-replacement solve has measured it already, unless it ran on the
  // Jacobi-scaled system
  if (!jac && h->known_true >= 0.0 && (rc == BCG_OK || rc == BCG_NOT_CONVERGED)) {
    h->info.true_rel_res = h->known_true;
  } else if (rc != BCG_EINVAL && rc != BCG_EHIP && rc != BCG_ENOMEM && (int)h->ref_r0.size() == h->k) {
    launch_residual(h->pl, h->rowptr, h->colind, h->vals, B, X, h->Q, nullptr, h->partN, 0, h->stream);
    launch_reduce(h->pl, h->partN, h->rnew, h->pl.W, nullptr, h->stream);
    std::vector<double> n2;
    if (fetch_norms(h, h->rnew, n2) == BCG_OK) h->info.true_rel_res = max_ratio(n2, jac ? h->true_r0 : h->ref_r0);
  }
  double m = 0.0;
  for (double v : h->host_ratios) m = std::max(m, v);
  h->info.max_rel_res = m;
  if (mixed) h->info.max_rel_res = h->info.true_rel_res;
  h->info.status = rc;
  h->info.converged = rc == BCG_OK;
  h->info.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return rc;
}

int bcg_update_values(bcg_handle* h, const double* values) {
  if (!h || !values) return fail(BCG_EINVAL, "handle and values must be non-NULL");
  DeviceGuard g(h->device);
  HIP_TRY(hipMemcpyAsync(h->vals, values, sizeof(double) * h->nnz, hipMemcpyDeviceToDevice, h->stream));
  launch_cast_values(h->nnz, h->vals, h->vals32, h->stream);
  HIP_TRY(hipGetLastError());
  if (h->precond == BCG_PRECOND_JACOBI) {
    const int rc = jacobi_prepare(h);
    if (rc) {
      h->precond = BCG_PRECOND_NONE;
      return rc;
    }
  }
  return BCG_OK;
}

int bcg_set_preconditioner(bcg_handle* h, int kind) {
  if (!h) return fail(BCG_EINVAL, "handle is NULL");
  if (kind != BCG_PRECOND_NONE && kind != BCG_PRECOND_JACOBI) return fail(BCG_EINVAL, "unknown preconditioner %d", kind);
  DeviceGuard g(h->device);
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->precond = BCG_PRECOND_NONE;
  if (kind == BCG_PRECOND_NONE) return BCG_OK;
  const int rc = jacobi_prepare(h);
  if (rc) return rc;
  h->precond = BCG_PRECOND_JACOBI;
  return BCG_OK;
}

int bcg_csr_outer(bcg_handle* h, const double* Y, const double* X, double alpha, double* out_vals) {
  if (!h || !Y || !X || !out_vals) return fail(BCG_EINVAL, "NULL argument");
  DeviceGuard g(h->device);
  launch_sampled_outer(h->n, h->k, h->rowptr, h->colind, Y, X, alpha, out_vals, h->stream);
  HIP_TRY(hipGetLastError());
  return BCG_OK;
}

int bcg_set_profiling(bcg_handle* h, int enable) {
  if (!h) return fail(BCG_EINVAL, "handle is NULL");
  DeviceGuard g(h->device);
  HIP_TRY(hipStreamSynchronize(h->stream));
  prof_collect(h, -1);  // drop anything pending
  if (enable)
    for (auto& t : h->prof) t = bcg_kernel_time{0, 0.0};
  h->prof_on = enable != 0;
  h->prof_mask = static_cast<unsigned>(enable);
  return BCG_OK;
}

int bcg_get_kernel_times(const bcg_handle* h, bcg_kernel_time* out, int count) {
  if (!h || !out || count < 0) return fail(BCG_EINVAL, "NULL argument");
  for (int i = 0; i < count && i < BCG_NUM_KERNEL_CLASSES; ++i) out[i] = h->prof[i];
  return BCG_OK;
}

int bcg_set_row_schedule(bcg_handle* h, const int32_t* order) {
  if (!h) return fail(BCG_EINVAL, "handle is NULL");
  DeviceGuard g(h->device);
  HIP_TRY(hipStreamSynchronize(h->stream));
  if (!order) {
    h->pl.sched = nullptr;
    return rebuild_sell(h);
  }
  int rc;
  if (!h->sched && (rc = dalloc(&h->sched, h->n))) return rc;
  HIP_TRY(hipMemcpyAsync(h->sched, order, sizeof(int32_t) * h->n, hipMemcpyDeviceToDevice, h->stream));
  // permutation check (memory safety of the product, and every row of Q
  // written once); the row counters borrow the workspace of Q, the flag lives
  // in the state
  DevState z{};
  HIP_TRY(hipMemcpyAsync(h->st, &z, sizeof z, hipMemcpyHostToDevice, h->stream));
  int* seen = reinterpret_cast<int*>(h->Q);
  HIP_TRY(hipMemsetAsync(seen, 0, sizeof(int) * h->n, h->stream));
  launch_check_perm(h->sched, h->n, seen, &h->st->status, h->stream);
  HIP_TRY(hipGetLastError());
  DevState out{};
  if ((rc = read_state(h, &out))) return rc;
  if (out.status != 0) {
    h->pl.sched = nullptr;
    (void)rebuild_sell(h);  // the SELL copy follows the natural order too
    return fail(BCG_EINVAL, "row schedule is not a permutation of 0..n-1");
  }
  h->pl.sched = h->sched;
  return rebuild_sell(h);
}

int bcg_set_sell(bcg_handle* h, int enable, int sigma) {
  if (!h) return fail(BCG_EINVAL, "handle is NULL");
  if (enable && (sigma < 1 || (sigma > 1 && sigma % 16 != 0)))
    return fail(BCG_EINVAL, "sigma must be 1 or a multiple of 16 (got %d)", sigma);
  DeviceGuard g(h->device);
  HIP_TRY(hipStreamSynchronize(h->stream));
  h->sell = 0;
  free_sell(h);
  if (!enable) return BCG_OK;
  h->sell_sigma = sigma;
  const int rc = build_sell(h);
  if (rc) {
    free_sell(h);
    return rc;
  }
  h->sell = 1;
  return BCG_OK;
}

int64_t bcg_sell_layout(int64_t n, const int32_t* rowptr, const int32_t* colind, const int32_t* order, int sigma,
                        int32_t* slice_ptr, int32_t* perm, int32_t* col, int32_t* map) {
  g_error.clear();
  if (n < 1 || n >= INT32_MAX || !rowptr) return fail(BCG_EINVAL, "n must be in [1, 2^31 - 1) and rowptr non-NULL");
  if (sigma < 1 || (sigma > 1 && sigma % 16 != 0))
    return fail(BCG_EINVAL, "sigma must be 1 or a multiple of 16 (got %d)", sigma);
  if (rowptr[0] != 0) return fail(BCG_EINVAL, "rowptr[0] must be 0");
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return fail(BCG_EINVAL, "rowptr decreases at row %lld", (long long)i);
  if (rowptr[n] > 0 && !colind) return fail(BCG_EINVAL, "colind must be non-NULL");
  if (order)
    for (int64_t i = 0; i < n; ++i)
      if (order[i] < 0 || order[i] >= n) return fail(BCG_EINVAL, "order has entries outside [0, n)");
  std::vector<int32_t> sp, pm, cl, mp;
  const int rc = sell_layout_host(n, rowptr, colind, order, sigma, sp, pm, cl, mp);
  if (rc) return rc;
  const int64_t ns = (n + 15) / 16, slots = sp[ns];
  if (!slice_ptr) return slots;
  if (!perm || !col || !map) return fail(BCG_EINVAL, "perm, col and map must be non-NULL with slice_ptr");
  std::memcpy(slice_ptr, sp.data(), sizeof(int32_t) * (ns + 1));
  std::memcpy(perm, pm.data(), sizeof(int32_t) * ns * 16);
  std::memcpy(col, cl.data(), sizeof(int32_t) * slots);
  std::memcpy(map, mp.data(), sizeof(int32_t) * slots);
  return slots;
}

int bcg_get_info(const bcg_handle* h, bcg_info* info) {
  if (!h || !info) return fail(BCG_EINVAL, "NULL argument");
  *info = h->info;
  return BCG_OK;
}

int bcg_get_column_ratios(const bcg_handle* h, double* ratios, int k) {
  if (!h || !ratios || k != h->k) return fail(BCG_EINVAL, "ratios must hold exactly k values");
  std::memcpy(ratios, h->host_ratios.data(), sizeof(double) * k);
  return BCG_OK;
}

}  // extern "C"
