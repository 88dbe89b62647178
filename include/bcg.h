/*
 * bcg.h -- C ABI of the MI355X (gfx950) block Conjugate Gradients library.
 *
 * Solves A X = B for a sparse symmetric positive definite A (n x n, CSR) and
 * k right-hand sides (Dreier & Engwer, "Strategies for the vectorized Block
 * Conjugate Gradients method", Section 1 problem statement), with the
 * stabilised block CG of Algorithm 1 (Section 3) and the preconditioner
 * M = I, over one of the *-subalgebras of Section 2:
 *
 *   BCG_BLOCK    classical block CG, S = R^{k x k}             (p = k)
 *   BCG_GLOBAL   S = R^{p x p} (x) I_q, one p x p coefficient shared by the
 *                q = k/p contiguous column groups              (p | k)
 *   BCG_PARALLEL S = diag(R^k), k independent CGs in lockstep  (p = 1)
 *   BCG_HYBRID   S = diag(R^{p x p}, ..., R^{p x p}), q independent
 *                p-column block CGs                            (p | k)
 *
 * Memory, layout and ownership
 *   - Every array argument is a DEVICE pointer on the GPU that was current
 *     when the handle was created, unless a comment says "host".
 *   - Block vectors (B, X, Y, G) are n x k, row-major, k fastest (element
 *     (i, j) at offset i*k + j), FP64. This is the paper's layout with the
 *     right-hand-side index innermost (Section 4).
 *   - CSR: rowptr int32[n+1] (rowptr[0] = 0, non-decreasing, rowptr[n] = nnz),
 *     colind int32[nnz] in [0, n), values FP64[nnz]. Indices are int32, so
 *     nnz must be below 2^31.
 *   - bcg_create copies the CSR into library-owned device memory (plus an FP32
 *     copy of the values); the caller may free its arrays afterwards. The
 *     handle owns its workspace (residual, search directions, products,
 *     reduction partials), allocated at create (and, for the FP32-refinement
 *     mode, on the first solve in that mode).
 *   - Caller-owned arrays are borrowed for the duration of a call only.
 *
 * Streams and synchronisation
 *   - All device work of a handle is enqueued on the stream given to
 *     bcg_set_stream (default: the null stream). bcg_solve returns only after
 *     its work on that stream has finished. The other calls taking device
 *     pointers are stream-ordered and return after enqueueing.
 *   - A handle is not thread-safe; distinct handles are independent.
 *
 * Errors
 *   - Calls return a status code (BCG_OK = 0; negative = error). The text of
 *     the last error of the calling thread is returned by bcg_last_error().
 */
#ifndef BCG_H
#define BCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define BCG_OK 0
#define BCG_NOT_CONVERGED 1 /* maxit reached; X holds the last iterate */
#define BCG_EINVAL (-1)     /* invalid argument or input (see each call)  */
#define BCG_EBREAKDOWN (-2) /* numerical breakdown; X holds the last iterate */
#define BCG_ENOMEM (-3)     /* device allocation failed */
#define BCG_EHIP (-4)       /* HIP runtime error */

typedef enum {
  BCG_BLOCK = 0,
  BCG_GLOBAL = 1,
  BCG_PARALLEL = 2,
  BCG_HYBRID = 3
} bcg_subalgebra;

typedef enum {
  BCG_FP64 = 0,         /* everything in FP64 */
  BCG_FP32_REFINE = 1,  /* FP32 inner block CG (FP64 block products and small
                           solves), FP64 outer iterative refinement; each
                           outer step restarts the inner iteration */
  BCG_FP32_RELIABLE = 2 /* the same FP32 iteration kept running across the
                           FP64 corrections: residual replacement (reliable
                           updates) instead of restarts */
} bcg_precision;

typedef struct bcg_handle bcg_handle;

/* Sparse matrix in CSR form (device pointers; see the layout notes above). */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int32_t *rowptr;
  const int32_t *colind;
  const double *values;
} bcg_csr;

/* Result summary of the last bcg_solve (host struct). */
typedef struct {
  int32_t status;           /* return value of the last bcg_solve */
  int32_t iterations;       /* products A*P, summed over inner solves */
  int32_t outer_iterations; /* refinement steps (0 in FP64 mode) */
  int32_t converged;        /* 1 if the stop rule was met */
  int32_t fp64_fallback;    /* refinement stagnated and finished in FP64 */
  int32_t k;
  double max_rel_res;       /* max_j ||R_j|| / ||R0_j|| at exit: the recursive
                               residual (FP64 mode) or the FP64 true residual
                               (refinement mode) */
  double true_rel_res;      /* max_j ||(B - A X)_j|| / ||R0_j|| after the
                               solve, recomputed in FP64 */
  double solve_ms;          /* wall time spent inside bcg_solve */
} bcg_info;

/*
 * bcg_create -- build a solver for A with k right-hand sides.
 *   A           CSR of an SPD matrix (device arrays, copied).
 *   k           1 <= k <= 256.
 *   subalgebra  one of bcg_subalgebra.
 *   p           block size: BLOCK p in {0, k}; PARALLEL p in {0, 1};
 *               GLOBAL p = 0 (means 1) or 1 <= p <= k with k % p == 0;
 *               HYBRID 1 <= p <= k with k % p == 0.
 *   out         host pointer receiving the new handle.
 * Returns BCG_EINVAL for invalid n, nnz, k, subalgebra or p, and for
 * malformed CSR contents: rowptr[0] != 0, a decreasing rowptr, rowptr[n] !=
 * nnz, or a column index outside [0, n). The contents are checked on the
 * device after the copy and before any kernel reads a row range, so a
 * malformed matrix is rejected instead of driving a gather out of bounds.
 * Symmetry and definiteness remain the caller's contract (a matrix without
 * them can end a solve in BCG_EBREAKDOWN). BCG_ENOMEM, BCG_EHIP otherwise.
 * Section 2 (subalgebra definitions) fixes the admissible p.
 */
int bcg_create(const bcg_csr *A, int k, int subalgebra, int p, bcg_handle **out);

/* Releases the handle and everything it owns. NULL is ignored. */
void bcg_destroy(bcg_handle *h);

/* Sets the HIP stream (a hipStream_t, e.g. torch's current stream) used by
 * every later call on this handle. NULL selects the null stream. */
int bcg_set_stream(bcg_handle *h, void *hip_stream);

/*
 * bcg_set_precision -- choose FP64 or FP32 inner solves with FP64 refinement.
 * BCG_FP32_REFINE (restarted inner solves):
 *   inner_tol    depth of the inner FP32 solves: each asks for the remaining
 *                reduction 0.5 tol / ratio, but no deeper than inner_tol / 4
 *                (0 <= inner_tol < 1; 0 selects 4e-6 for groups of p <= 16
 *                and 1e-4 for wider ones, where FP32 block iterates lose
 *                accuracy sooner).
 *   inner_maxit  iteration cap of each inner solve (>= 1; default 1000).
 *   max_outer    cap on refinement steps (>= 1; default 50).
 * BCG_FP32_RELIABLE (residual replacement):
 *   inner_tol    replacement threshold delta: the FP64 correction and
 *                residual replacement happen whenever the FP32 recursive
 *                residual has fallen to delta times its value at the last
 *                correction, or to tol (0 <= delta < 1; 0 selects 1e-2 for
 *                groups of p <= 16 and 1e-1 for wider ones).
 *   inner_maxit  cap on FP32 iterations between two corrections.
 *   max_outer    cap on corrections.
 *   After a correction X += s D, R = B - A X (FP64), s' = max_j ||R_j||,
 *   the iteration continues on the scaled system with R32 = R / s', its
 *   search direction P32 *= s / s' and the last line-6 product rho *=
 *   (s / s')^2, from line 10 (residual replacement: van der Vorst and Ye,
 *   SIAM J. Sci. Comput. 22 (2000); reliable updates: Sleijpen and van der
 *   Vorst, Computing 56 (1996)).
 * Both forms stop on the FP64 true residual, and finish with the FP64
 * iteration from the current X if a correction fails to halve the largest
 * relative residual (bcg_info.fp64_fallback). Not in the paper: the
 * mixed-precision forms keep the block products, the Cholesky and LU
 * solves and the true residual in FP64.
 */
int bcg_set_precision(bcg_handle *h, int mode, double inner_tol, int inner_maxit, int max_outer);

/*
 * bcg_solve -- run Algorithm 1 (M = I) on A X = B.
 *   B      n x k right-hand sides (read).
 *   X      n x k initial guess on entry, solution on exit (read/write; may
 *          not alias B).
 *   tol    stop when every column's residual norm fell below tol times its
 *          initial residual norm (Section 4 stop rule, 2-norm of the
 *          recursive residual, checked after the residual update). tol = 0
 *          runs exactly maxit iterations.
 *   maxit  iteration cap (>= 0); in refinement mode the cap of each FP64
 *          fallback.
 * Returns BCG_OK (converged, or B - A X0 = 0), BCG_NOT_CONVERGED,
 * BCG_EINVAL (non-finite B or X0, or a zero initial-residual column in a
 * subalgebra other than the diagonal one: PARALLEL, or HYBRID with p = 1),
 * BCG_EBREAKDOWN (a Cholesky pivot of the symmetrised alpha not above
 * p*eps times its diagonal, a zero LU pivot of rho, or a non-finite
 * residual), BCG_EHIP. Synchronous with respect to the handle's stream.
 */
int bcg_solve(bcg_handle *h, const double *B, double *X, double tol, int maxit);

/*
 * bcg_solve_noalloc -- bcg_create + bcg_solve (FP64, M = I, natural row
 * order) + bcg_destroy in one call that allocates no memory: for callers
 * that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Arguments as bcg_create and bcg_solve;
 * hip_stream as bcg_set_stream; info (host, may be NULL) receives what
 * bcg_get_info would report.
 *   - The matrix is read in place from the caller's arrays (not copied);
 *     its contents are checked on the device first, as bcg_create does.
 *   - Every workspace buffer of the solve (residual, search directions,
 *     products, reduction partials, coefficients, device state) lives in
 *     one fixed array of 128 MiB that each GPU the library runs on holds
 *     until the process ends. A solve whose workspace (3 n k doubles plus
 *     the partial products) exceeds it returns BCG_EINVAL with a message;
 *     bcg_create then serves it.
 *   - The array keeps the last call's contents: each call resets the
 *     device state it reads. Calls that overlap on one GPU (other threads,
 *     other streams) share the array and race; the caller serialises them.
 *   - Results equal bcg_solve's for the same inputs (same kernels, same
 *     launch plan). The solve reads its state back synchronously after each
 *     chunk of iterations (no pinned memory or events), so it can be slower
 *     than a handle's solve on long iteration counts.
 * Returns as bcg_solve, and BCG_EINVAL for malformed CSR, k, subalgebra or
 * p, or a workspace beyond the fixed array.
 */
int bcg_solve_noalloc(const bcg_csr *A, int k, int subalgebra, int p, const double *B, double *X, double tol,
                      int maxit, void *hip_stream, bcg_info *info);

/* Copies new matrix values (same pattern as at create; device array of nnz
 * FP64) into the handle, e.g. for a differentiable solve. Stream-ordered;
 * with the Jacobi preconditioner on, also recomputes its scaling and waits
 * for it (BCG_EINVAL, and the preconditioner off, if the new diagonal is
 * not positive). */
int bcg_update_values(bcg_handle *h, const double *values);

/*
 * bcg_set_preconditioner -- the preconditioner M of Algorithm 1 (lines 2,
 * 10, 11 and 13). kind: BCG_PRECOND_NONE (M = I, the default) or
 * BCG_PRECOND_JACOBI (M = diag(A)). Jacobi runs block CG on the
 * symmetrically scaled system D^{-1/2} A D^{-1/2} Y = D^{-1/2} B, X =
 * D^{-1/2} Y, whose iterates are those of Algorithm 1 with M = diag(A); the
 * stop rule then compares the M^{-1}-norms sqrt(R_j^T M^{-1} R_j) of the
 * recursive residual columns with their initial values (info.max_rel_res,
 * bcg_get_column_ratios), while info.true_rel_res stays the Euclidean
 * ||B - A X||_j / ||B - A X0||_j. Needs a positive finite diagonal entry in
 * every row: BCG_EINVAL otherwise (preconditioner left off). The handle
 * keeps n scale factors and scaled FP64 and FP32 copies of the values, and
 * from the first solve on an n x k FP64 block for the scaled B; B itself is
 * not modified, X is scaled in place during the solve. Synchronous.
 */
enum { BCG_PRECOND_NONE = 0, BCG_PRECOND_JACOBI = 1 };
int bcg_set_preconditioner(bcg_handle *h, int kind);

/*
 * bcg_csr_outer -- sampled outer product on the pattern of A:
 *   out_vals[e] = alpha * sum_c Y[row(e), c] * X[col(e), c], e < nnz.
 * With Y = A^{-1} G and alpha = -1 this is dL/d(values of A) for a loss
 * with dL/dX = G (adjoint of the solve). Y, X: n x k FP64; out_vals: FP64[nnz]
 * (written, not accumulated). Stream-ordered.
 */
int bcg_csr_outer(bcg_handle *h, const double *Y, const double *X, double alpha, double *out_vals);

/*
 * bcg_set_row_schedule -- optional processing order of the rows in the
 * sparse product Q = A P (not in the paper: a cache-locality schedule; the
 * paper observes the product's cache behaviour degrading for large k,
 * Section 4). order: device int32[n], a permutation of 0..n-1, copied.
 * Every row is computed exactly as before; only the order, and with it the
 * reuse of gathered rows of P in cache, changes (and the rounding order of
 * the partial alpha products). NULL restores the natural order. An order
 * that is not a permutation (an entry outside [0, n), or a row listed twice)
 * returns BCG_EINVAL and leaves the natural order. Synchronous.
 */
int bcg_set_row_schedule(bcg_handle *h, const int32_t *order);

/*
 * bcg_set_sell -- keep a SELL-C-sigma copy of the matrix (sliced ELLPACK,
 * C = 16 rows per slice, rows sorted by decreasing length within windows of
 * sigma consecutive rows; Section 4 names this format as the remedy for the
 * sparse product's cache behaviour for wide blocks) and run the matrix-core
 * sparse product on it. The rows are taken in the current row schedule
 * (natural order without one); a later bcg_set_row_schedule rebuilds the
 * copy. Every row of Q = A P is computed from the same entries in the same
 * order as from CSR; with sigma = 1 the positions of the rows do not move,
 * and a solve is bitwise the same as with CSR. Padding slots hold value 0 and
 * the row's own column.
 * enable: 1 builds (or rebuilds) the copy, 0 frees it. sigma: 1 (no
 * sorting) or a multiple of 16. The layout is built on the host from a copy
 * of the pattern; the values are taken from the handle's current values
 * (after bcg_update_values and the Jacobi scaling) at the start of every
 * solve. Solves whose row kernels are not the matrix-core ones (k not a
 * multiple of 16, p outside the supported set, X not 16-byte aligned) use
 * the CSR product. Storage: 4 (n/16 + 1) + 4 n + 20 s bytes for s padded
 * slots. Errors: BCG_EINVAL for a bad sigma or more than 2^31 - 1 slots,
 * BCG_ENOMEM, BCG_EHIP. Synchronous.
 */
int bcg_set_sell(bcg_handle *h, int enable, int sigma);

/*
 * bcg_sell_layout -- the SELL-16-sigma layout that bcg_set_sell stores,
 * computed from a CSR pattern on the host (no device work; for callers that
 * inspect or reuse the layout, and for tests). All pointers are HOST arrays.
 *   rowptr int32[n+1] (rowptr[0] = 0, non-decreasing), colind int32[rowptr[n]],
 *   order int32[n] with entries in [0, n), or NULL for the natural order.
 * Positions follow `order`; within each window of sigma positions the rows are
 * sorted by decreasing length (stable). Slice S holds positions 16 S .. 16 S +
 * 15 (positions past n repeat the last position's row) and has width w = the
 * longest row length among its real positions, at least 1. Slot t of position
 * 8 h + r of slice S (h in {0, 1}, r < 8) is entry
 *   slice_ptr[S] + 8 w h + 8 t + r
 * of col and map: the row's t-th CSR column and entry index, or for padding the
 * row itself and -1.
 * With slice_ptr NULL only the slot count is returned. Otherwise slice_ptr
 * (ceil(n/16) + 1 entries), perm (16 ceil(n/16): position -> row), col and
 * map (slot count entries each) are written.
 * Returns the slot count, or BCG_EINVAL for a bad argument (sigma not 1 or a
 * multiple of 16, a malformed rowptr, order out of range, more than 2^31 - 1
 * slots).
 */
int64_t bcg_sell_layout(int64_t n, const int32_t *rowptr, const int32_t *colind, const int32_t *order, int sigma,
                        int32_t *slice_ptr, int32_t *perm, int32_t *col, int32_t *map);

/* Copies the summary of the last solve into *info (host struct). */
int bcg_get_info(const bcg_handle *h, bcg_info *info);

/* Copies the k per-column final ratios ||R_j|| / ||R0_j|| of the last solve
 * into host array ratios[k]. */
int bcg_get_column_ratios(const bcg_handle *h, double *ratios, int k);

/*
 * Per-kernel-class timing (not in the paper; measurement support). When
 * enabled, HIP events are recorded on the handle's stream around every
 * launch, and the durations of launches that did work (iterations up to the
 * one the stop rule accepted; launches that returned at entry after the stop
 * are excluded) are accumulated per class until profiling is enabled again.
 */
enum {
  BCG_K_SPMM = 0,      /* Q = A P with the partial <<P, Q>>              */
  BCG_K_UPDATE_R = 1,  /* R -= Q lambda with <<R, R>> and column norms   */
  BCG_K_UPDATE_XP = 2, /* X += P lambda, P = R + P beta, partial <<P, R>> */
  BCG_K_REDUCE = 3,    /* fixed-order sums of partials outside the loop  */
  BCG_K_SMALL = 4,     /* per-iteration sums of the partials with the
                          Cholesky / LU solves and the stop rule they feed */
  BCG_K_RESIDUAL = 5,  /* B - A X, FP32 start of a refinement step, X += s D */
  BCG_K_PRODUCT = 6,   /* stand-alone block products (large p)           */
  BCG_NUM_KERNEL_CLASSES = 7
};

typedef struct {
  int64_t launches; /* counted launches */
  double total_ms;  /* summed event-measured durations */
} bcg_kernel_time;

/* enable: bit mask of classes to record (1 << BCG_K_*; -1 = all); a non-zero
 * mask resets the counters and starts recording, 0 stops. */
int bcg_set_profiling(bcg_handle *h, int enable);

/* Copies min(count, BCG_NUM_KERNEL_CLASSES) classes into out (host). */
int bcg_get_kernel_times(const bcg_handle *h, bcg_kernel_time *out, int count);

/* Text of the calling thread's last error ("" if none). Host string owned
 * by the library, valid until the next failing call on this thread. */
const char *bcg_last_error(void);

/*
 * Stencil matrices (the paper's test problem class, Section 4: heterogeneous
 * Poisson with a 5-point finite-difference stencil; 7-point in 3D).
 * Interior grid of N^dim points, Dirichlet neighbours eliminated,
 * lexicographic order with x fastest, ascending columns per row. Without
 * coefficients: 2*dim on the diagonal, -1 off it. With per-cell coefficients
 * kappa (FP64[N^dim]): interior face value ((2*ka)*kb)/(ka+kb), boundary
 * face value kappa of the cell, off-diagonal -face, diagonal = sum of the
 * cell's face values in the order x-, x+, y-, y+, z-, z+ (IEEE FP64, each
 * operation rounded once).
 */

/* Number of stored entries, (2*dim+1)*N^dim - 2*dim*N^(dim-1), or -1 for
 * dim not in {2, 3}, N < 1, or nnz / n beyond int32. Host-only. */
int64_t bcg_stencil_nnz(int dim, int N);

/* Writes rowptr int32[n+1], colind int32[nnz], values FP64[nnz] (device,
 * caller-allocated). kappa may be NULL (constant coefficient 1). Stream-
 * ordered on hip_stream (NULL = null stream). */
int bcg_stencil_build(int dim, int N, const double *kappa, int32_t *rowptr, int32_t *colind,
                      double *values, void *hip_stream);

/* Row schedule for bcg_set_row_schedule on the stencil matrices: in 3D,
 * x-y tiles of tile x tile cells in row-major tile order, each swept through
 * all z planes (x fastest inside a tile), so the z-neighbours a row gathers
 * were touched one plane earlier; in 2D the natural order. order: device
 * int32[N^dim]. Stream-ordered. */
int bcg_stencil_schedule(int dim, int N, int tile, int32_t *order, void *hip_stream);

/* Brick row schedule of the 3D stencil on an N^3 grid (not in the paper: a
 * cache-locality order for wide blocks, where a row of P spans several
 * cache lines): tiles of tile[0] x tile[1] x tile[2] cells (x, y, z) visited
 * tile column by tile column (row-major over the tiles' y, x) and each
 * column swept through z; inside a tile, bricks of brick[0] x brick[1] x
 * brick[2] cells with x fastest, then y, then z; inside a brick x fastest.
 * A 16-row step of the sparse product is then a compact brick, so fewer
 * distinct neighbour rows are gathered per step. tile, brick: host int[3]
 * with brick[d] | tile[d] | N. order: device int32[N^3], position -> row.
 * Returns BCG_EINVAL for other sizes. Stream-ordered. */
int bcg_stencil_brick_schedule(int N, const int *tile, const int *brick, int32_t *order, void *hip_stream);

/* Transpose Jacobian of the stencil values with respect to kappa:
 * dkappa[c] = sum_e dvalues[e] * d values[e] / d kappa[c] (device arrays;
 * dvalues in the CSR order of bcg_stencil_build). Stream-ordered. */
int bcg_stencil_kappa_vjp(int dim, int N, const double *kappa, const double *dvalues,
                          double *dkappa, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* BCG_H */
