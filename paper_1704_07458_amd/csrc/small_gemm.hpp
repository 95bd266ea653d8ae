// FP64 products of the projected-problem sizes (n_s up to a few hundred) on
// MFMA: C = alpha op(A) op(B) + beta C, column-major.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lobpcg {

// Largest m, n, k the small-product kernel takes (callers use a library GEMM above).
constexpr int kSmallGemmMax = 2048;
inline bool small_dgemm_fits(int m, int n, int k) {
  return m <= kSmallGemmMax && n <= kSmallGemmMax && k <= kSmallGemmMax;
}

// op(A) is m x k (ta: A^T), op(B) is k x n (tb: B^T).  C must not overlap A or B.
// beta = 0 does not read C.
void small_dgemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A,
                 int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                 hipStream_t s);

// For each i < count: the diagonal blocks at off[i] of size dim[i] (dim[i] <=
// kSmallGemmMax): C(o:o+d, o:o+d) = A(o:o+d, o:o+d) B(o:o+d, o:o+d).  count <=
// kSmallGemmBatch.
constexpr int kSmallGemmBatch = 32;
void small_dgemm_diag_batch(int count, const int* off, const int* dim, const double* A, int64_t lda,
                            const double* B, int64_t ldb, double* C, int64_t ldc, hipStream_t s);

}  // namespace lobpcg
