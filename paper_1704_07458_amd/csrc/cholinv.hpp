// Cholesky factor and its inverse for the projected B-Gram matrix (one
// workgroup), used by the Rayleigh-Ritz step of Algorithm 7.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lobpcg {

// Largest n the one-workgroup kernel accepts.
int cholinv_max_n();

// In: A (column-major, lda >= n) symmetric, its upper triangle is read.
// Out: A = R, the upper Cholesky factor (R^T R = A, lower triangle zeroed);
// T (ldt >= n, must not overlap A) = R^-1 (upper, lower triangle zeroed);
// info[0] = 0, or j + 1 when the j-th pivot is not a finite positive number
// (A and T then hold partial results), info[1] = 0.  1 <= n <= cholinv_max_n().
void launch_cholinv_upper(int n, double* A, int64_t lda, double* T, int64_t ldt, int32_t* info,
                          hipStream_t s);

}  // namespace lobpcg
