// Stencil matrices of the paper's test problem class (Section 4: heterogeneous
// Poisson, 5-point finite differences; 7-point in 3D) built on the GPU, and
// the transpose Jacobian of their values with respect to the cell
// coefficients. Compiled with -ffp-contract=off: every face value is
// ((2*ka)*kb)/(ka+kb) with each operation rounded once, so the values match a
// plain IEEE FP64 evaluation bit for bit.
//
// Layout: interior unknowns c = x + N*y + N*N*z (x fastest), Dirichlet
// neighbours eliminated, columns ascending per row (z-, y-, x-, centre, x+,
// y+, z+). The row start of c has a closed form, so each thread writes its
// row without a prefix scan.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/bcg.h"

namespace {

constexpr int kThreads = 256;

struct Grid {
  int dim;
  int64_t N;
  int64_t n;
  int64_t stride[3];
};

// Number of c' in [0, c) whose coordinate with stride s equals v.
__device__ __forceinline__ int64_t count_coord(int64_t c, int64_t s, int64_t N, int64_t v) {
  const int64_t period = s * N;
  const int64_t full = c / period;
  const int64_t rem = c - full * period;
  int64_t part = rem - v * s;
  part = part < 0 ? 0 : (part > s ? s : part);
  return full * s + part;
}

// CSR offset of row c: (2*dim+1)*c minus the missing boundary neighbours of
// the rows before c.
__device__ __forceinline__ int64_t row_start(const Grid& g, int64_t c) {
  int64_t r = (2 * g.dim + 1) * c;
  for (int d = 0; d < g.dim; ++d)
    r -= count_coord(c, g.stride[d], g.N, 0) + count_coord(c, g.stride[d], g.N, g.N - 1);
  return r;
}

__device__ __forceinline__ double harmonic(double ka, double kb) { return ((2.0 * ka) * kb) / (ka + kb); }

__device__ __forceinline__ double kap(const double* kappa, int64_t c) { return kappa ? kappa[c] : 1.0; }

__global__ __launch_bounds__(kThreads) void k_build(Grid g, const double* __restrict__ kappa,
                                                    int32_t* __restrict__ rowptr, int32_t* __restrict__ colind,
                                                    double* __restrict__ values) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= g.n) return;
  int64_t x[3];
  for (int d = 0; d < g.dim; ++d) x[d] = (c / g.stride[d]) % g.N;
  const double kc = kap(kappa, c);
  double fm[3], fp[3];
  for (int d = 0; d < g.dim; ++d) {
    fm[d] = x[d] > 0 ? harmonic(kap(kappa, c - g.stride[d]), kc) : kc;
    fp[d] = x[d] < g.N - 1 ? harmonic(kc, kap(kappa, c + g.stride[d])) : kc;
  }
  double diag = fm[0];
  diag = diag + fp[0];
  for (int d = 1; d < g.dim; ++d) {
    diag = diag + fm[d];
    diag = diag + fp[d];
  }
  int64_t pos = row_start(g, c);
  rowptr[c] = static_cast<int32_t>(pos);
  if (c == g.n - 1) rowptr[g.n] = static_cast<int32_t>(row_start(g, g.n));
  for (int d = g.dim - 1; d >= 0; --d)
    if (x[d] > 0) {
      colind[pos] = static_cast<int32_t>(c - g.stride[d]);
      values[pos++] = -fm[d];
    }
  colind[pos] = static_cast<int32_t>(c);
  values[pos++] = diag;
  for (int d = 0; d < g.dim; ++d)
    if (x[d] < g.N - 1) {
      colind[pos] = static_cast<int32_t>(c + g.stride[d]);
      values[pos++] = -fp[d];
    }
}

// Position of each stored entry of row c, from its coordinates.
struct RowPos {
  int64_t start;
  int nminus;        // stored lower neighbours
  int minus_pos[3];  // offset of the -e_d neighbour in the row (if present)
  int plus_pos[3];   // offset of the +e_d neighbour (if present)
};

__device__ __forceinline__ RowPos row_pos(const Grid& g, int64_t c) {
  RowPos rp;
  rp.start = row_start(g, c);
  int64_t x[3];
  for (int d = 0; d < g.dim; ++d) x[d] = (c / g.stride[d]) % g.N;
  int o = 0;
  for (int d = g.dim - 1; d >= 0; --d)
    if (x[d] > 0) rp.minus_pos[d] = o++;
  rp.nminus = o++;  // centre
  for (int d = 0; d < g.dim; ++d)
    if (x[d] < g.N - 1) rp.plus_pos[d] = o++;
  return rp;
}

// dkappa[c] = sum over c's faces f of dL/dc_f * dc_f/dkappa_c, where an
// interior face appears as +c_f in both diagonals and -c_f in both
// off-diagonal entries, and a boundary face as +kappa_c in diag(c).
__global__ __launch_bounds__(kThreads) void k_kappa_vjp(Grid g, const double* __restrict__ kappa,
                                                        const double* __restrict__ dv, double* __restrict__ dk) {
  const int64_t c = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (c >= g.n) return;
  const RowPos rc = row_pos(g, c);
  const double dc = dv[rc.start + rc.nminus];
  const double kc = kappa[c];
  double acc = 0.0;
  for (int d = 0; d < g.dim; ++d) {
    const int64_t xd = (c / g.stride[d]) % g.N;
    for (int side = 0; side < 2; ++side) {
      const bool inside = side == 0 ? xd > 0 : xd < g.N - 1;
      if (!inside) {
        acc += dc;
        continue;
      }
      const int64_t nb = side == 0 ? c - g.stride[d] : c + g.stride[d];
      const RowPos rn = row_pos(g, nb);
      const double dnb = dv[rn.start + rn.nminus];
      const double d_cn = dv[rc.start + (side == 0 ? rc.minus_pos[d] : rc.plus_pos[d])];
      const double d_nc = dv[rn.start + (side == 0 ? rn.plus_pos[d] : rn.minus_pos[d])];
      const double w = dc + dnb - d_cn - d_nc;
      const double kn = kappa[nb];
      const double s = kc + kn;
      acc += w * (2.0 * kn * kn / (s * s));
    }
  }
  dk[c] = acc;
}

// order[e] = row of the e-th product row: x-y tiles of T x T cells in
// row-major tile order, each swept through all z planes, x fastest inside the
// tile (3D); the natural order in 2D.
__global__ __launch_bounds__(kThreads) void k_schedule(Grid g, int T, int32_t* __restrict__ order) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= g.n) return;
  if (g.dim != 3) {
    order[e] = static_cast<int32_t>(e);
    return;
  }
  const int64_t N = g.N;
  const int64_t ntx = (N + T - 1) / T;
  // tiles are visited in order; tile (ty, tx) holds w x h cells per plane
  int64_t rem = e, ty = 0, tx = 0;
  for (;;) {
    const int64_t w = min<int64_t>(T, N - tx * T), hgt = min<int64_t>(T, N - ty * T);
    const int64_t cells = w * hgt * N;
    if (rem < cells) {
      const int64_t z = rem / (w * hgt);
      const int64_t r = rem - z * (w * hgt);
      const int64_t y = ty * T + r / w, x = tx * T + r % w;
      order[e] = static_cast<int32_t>(x + N * y + N * N * z);
      return;
    }
    rem -= cells;
    if (++tx == ntx) {
      tx = 0;
      ++ty;
    }
  }
}

// Brick order of the 3D grid: tiles of tx x ty x tz cells, visited tile
// column by tile column (row-major over (ty, tx)), each column swept through
// z; inside a tile, bricks of bx x by x bz cells with x fastest, then y, then
// z; inside a brick, cells with x fastest. Position e -> row.
struct Bricks {
  int tx, ty, tz, bx, by, bz;
};
__global__ __launch_bounds__(kThreads) void k_brick_schedule(int64_t N, Bricks b, int32_t* __restrict__ order) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= N * N * N) return;
  const int64_t tv = (int64_t)b.tx * b.ty * b.tz, bv = (int64_t)b.bx * b.by * b.bz;
  const int64_t ntx = N / b.tx, ntz = N / b.tz, nbx = b.tx / b.bx, nby = b.ty / b.by;
  const int64_t t = e / tv, in_t = e - t * tv, br = in_t / bv, c = in_t - br * bv;
  const int64_t TZ = t % ntz, t2 = t / ntz, TX = t2 % ntx, TY = t2 / ntx;
  const int64_t BX = br % nbx, br2 = br / nbx, BY = br2 % nby, BZ = br2 / nby;
  const int64_t cx = c % b.bx, c2 = c / b.bx, cy = c2 % b.by, cz = c2 / b.by;
  const int64_t x = TX * b.tx + BX * b.bx + cx, y = TY * b.ty + BY * b.by + cy, z = TZ * b.tz + BZ * b.bz + cz;
  order[e] = static_cast<int32_t>(x + N * y + N * N * z);
}

bool make_grid(int dim, int N, Grid* g) {
  if ((dim != 2 && dim != 3) || N < 1) return false;
  g->dim = dim;
  g->N = N;
  g->n = 1;
  for (int d = 0; d < dim; ++d) {
    g->stride[d] = g->n;
    g->n *= N;
  }
  const int64_t nnz = (2 * dim + 1) * g->n - 2 * dim * (g->n / N);
  return g->n < INT32_MAX && nnz < INT32_MAX;
}

}  // namespace

extern "C" int64_t bcg_stencil_nnz(int dim, int N) {
  Grid g;
  if (!make_grid(dim, N, &g)) return -1;
  return (2 * dim + 1) * g.n - 2 * dim * (g.n / N);
}

extern "C" int bcg_stencil_build(int dim, int N, const double* kappa, int32_t* rowptr, int32_t* colind,
                                 double* values, void* hip_stream) {
  Grid g;
  if (!make_grid(dim, N, &g) || !rowptr || !colind || !values) return BCG_EINVAL;
  const int64_t blocks = (g.n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_build, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), g, kappa, rowptr, colind, values);
  return hipGetLastError() == hipSuccess ? BCG_OK : BCG_EHIP;
}

extern "C" int bcg_stencil_brick_schedule(int N, const int* tile, const int* brick, int32_t* order,
                                          void* hip_stream) {
  if (!tile || !brick || !order || N < 1 || static_cast<int64_t>(N) * N * N >= INT32_MAX) return BCG_EINVAL;
  for (int d = 0; d < 3; ++d)
    if (tile[d] < 1 || brick[d] < 1 || N % tile[d] != 0 || tile[d] % brick[d] != 0) return BCG_EINVAL;
  const Bricks b{tile[0], tile[1], tile[2], brick[0], brick[1], brick[2]};
  const int64_t n = static_cast<int64_t>(N) * N * N, blocks = (n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_brick_schedule, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), static_cast<int64_t>(N), b, order);
  return hipGetLastError() == hipSuccess ? BCG_OK : BCG_EHIP;
}

extern "C" int bcg_stencil_schedule(int dim, int N, int tile, int32_t* order, void* hip_stream) {
  Grid g;
  if (!make_grid(dim, N, &g) || tile < 1 || !order) return BCG_EINVAL;
  const int64_t blocks = (g.n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_schedule, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), g, tile, order);
  return hipGetLastError() == hipSuccess ? BCG_OK : BCG_EHIP;
}

extern "C" int bcg_stencil_kappa_vjp(int dim, int N, const double* kappa, const double* dvalues, double* dkappa,
                                     void* hip_stream) {
  Grid g;
  if (!make_grid(dim, N, &g) || !kappa || !dvalues || !dkappa) return BCG_EINVAL;
  const int64_t blocks = (g.n + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_kappa_vjp, dim3(static_cast<unsigned>(blocks)), dim3(kThreads), 0,
                     static_cast<hipStream_t>(hip_stream), g, kappa, dvalues, dkappa);
  return hipGetLastError() == hipSuccess ? BCG_OK : BCG_EHIP;
}
