// Jacobi preconditioning (M = diag(A)) by symmetric scaling: launchers of
// the set-up and per-solve scaling kernels (bcg_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bcg {

// dscale = diag(A)^{-1/2}; *flag = 1 where a diagonal entry is missing, not
// positive or not finite.
void launch_jacobi_scale(int64_t n, const int32_t* rowptr, const int32_t* colind, const double* vals, double* dscale,
                         int* flag, hipStream_t s);
// Values of D^{-1/2} A D^{-1/2}, FP64 and FP32.
void launch_scale_values(int64_t n, const int32_t* rowptr, const int32_t* colind, const double* vals,
                         const double* dscale, double* vs, float* vs32, hipStream_t s);
// dst = D^{-1/2} src (divide = 0) or D^{1/2} src (divide = 1) for a row-major
// n x k block; dst may be src.
void launch_scale_rows(int64_t n, int k, const double* src, const double* dscale, double* dst, int divide,
                       hipStream_t s);

}  // namespace bcg
