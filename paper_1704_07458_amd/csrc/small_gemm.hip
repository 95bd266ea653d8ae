// FP64 MFMA products for the projected problems (sizes of a few hundred): one
// 256-thread workgroup per 16 x 16 block of C, the four waves taking every
// fourth 4-deep slice of K (v_mfma_f64_16x16x4f64), their partial blocks summed
// through LDS in wave order (deterministic).  A library GEMM picks 64- or
// 128-wide tiles for these shapes and leaves most of the chip idle; here a
// 330 x 330 product spreads over 441 workgroups.
#include "small_gemm.hpp"

#include <hip/hip_runtime.h>

#include "common.hpp"

namespace lobpcg {
namespace {

constexpr int kWave = 64;
constexpr int kSgWaves = 4;
constexpr int kSgPre = 4;  // slices loaded ahead of the products

typedef double v4d __attribute__((ext_vector_type(4)));

struct SgBatch {
  int off[kSmallGemmBatch];
  int dim[kSmallGemmBatch];
};

// MFMA 16x16x4 f64 lane layout: A (16 x 4) lane l holds A[l % 16][l / 16],
// B (4 x 16) lane l holds B[l / 16][l % 16], D (16 x 16) lane l element q holds
// D[l / 16 + 4 q][l % 16].
template <bool TA, bool TB>
__global__ __launch_bounds__(kSgWaves * kWave) void small_dgemm_kernel(
    int m, int n, int k, double alpha, const double* __restrict__ A, int64_t lda,
    const double* __restrict__ B, int64_t ldb, double beta, double* __restrict__ C, int64_t ldc,
    int tiles_m, SgBatch batch, int batched) {
  __shared__ double red[kSgWaves - 1][4][kWave];
  if (batched) {
    const int o = batch.off[blockIdx.z], d = batch.dim[blockIdx.z];
    m = n = k = d;
    A += o + (int64_t)o * lda;
    B += o + (int64_t)o * ldb;
    C += o + (int64_t)o * ldc;
  }
  const int tm = blockIdx.x % tiles_m, tn = blockIdx.x / tiles_m;
  const int i0 = tm * 16, j0 = tn * 16;
  if (i0 >= m || j0 >= n) return;  // a whole workgroup (batched blocks differ in size)
  const int t = threadIdx.x;
  const int wave = t / kWave, lane = t % kWave;
  const int li = lane % 16, lk = lane / 16;
  const int ia = i0 + li, jb = j0 + li;
  const bool oka = ia < m, okb = jb < n;
  // element (row r, depth kk) of op(A) and (depth kk, column c) of op(B)
  auto ga = [&](int kk) -> double {
    if (!oka || kk >= k) return 0.0;
    return TA ? A[kk + (int64_t)ia * lda] : A[ia + (int64_t)kk * lda];
  };
  auto gb = [&](int kk) -> double {
    if (!okb || kk >= k) return 0.0;
    return TB ? B[jb + (int64_t)kk * ldb] : B[kk + (int64_t)jb * ldb];
  };
  const int nks = (k + 3) / 4;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  // slices wave, wave + 4, ...; kSgPre of them loaded ahead
  double pa[kSgPre], pb[kSgPre];
#pragma unroll
  for (int u = 0; u < kSgPre; ++u) {
    const int kk = 4 * (wave + kSgWaves * u) + lk;
    pa[u] = ga(kk);
    pb[u] = gb(kk);
  }
  for (int ks = wave; ks < nks; ks += kSgWaves * kSgPre) {
#pragma unroll
    for (int u = 0; u < kSgPre; ++u) {
      const double a = pa[u], b = pb[u];
      const int kk = 4 * (ks + kSgWaves * (u + kSgPre)) + lk;
      pa[u] = ga(kk);
      pb[u] = gb(kk);
      if (ks + kSgWaves * u < nks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) red[wave - 1][q][lane] = acc[q];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      double v = acc[q];
#pragma unroll
      for (int w = 0; w < kSgWaves - 1; ++w) v += red[w][q][lane];
      const int i = i0 + lk + 4 * q, j = j0 + li;
      if (i < m && j < n) {
        double* c = C + i + (int64_t)j * ldc;
        *c = beta == 0.0 ? alpha * v : fma(alpha, v, beta * *c);
      }
    }
  }
}

template <bool TA, bool TB>
void launch(int m, int n, int k, double alpha, const double* A, int64_t lda, const double* B,
            int64_t ldb, double beta, double* C, int64_t ldc, const SgBatch& batch, int count,
            hipStream_t s) {
  const int tiles_m = (m + 15) / 16, tiles_n = (n + 15) / 16;
  hipLaunchKernelGGL((small_dgemm_kernel<TA, TB>), dim3((unsigned)(tiles_m * tiles_n), 1,
                     (unsigned)(count > 0 ? count : 1)), dim3(kSgWaves * kWave), 0, s, m, n, k,
                     alpha, A, lda, B, ldb, beta, C, ldc, tiles_m, batch, count > 0 ? 1 : 0);
  LOBPCG_HIP(hipGetLastError());
}

}  // namespace

void small_dgemm(bool ta, bool tb, int m, int n, int k, double alpha, const double* A,
                 int64_t lda, const double* B, int64_t ldb, double beta, double* C, int64_t ldc,
                 hipStream_t s) {
  if (m == 0 || n == 0) return;
  LOBPCG_CHECK(small_dgemm_fits(m, n, k) && m > 0 && n > 0 && k >= 0, LOBPCG_ERR_ARG,
               "small_dgemm: sizes out of range");
  SgBatch none{};
  if (ta) {
    if (tb) launch<true, true>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, none, 0, s);
    else launch<true, false>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, none, 0, s);
  } else {
    if (tb) launch<false, true>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, none, 0, s);
    else launch<false, false>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, none, 0, s);
  }
}

void small_dgemm_diag_batch(int count, const int* off, const int* dim, const double* A, int64_t lda,
                            const double* B, int64_t ldb, double* C, int64_t ldc, hipStream_t s) {
  LOBPCG_CHECK(count >= 0 && count <= kSmallGemmBatch, LOBPCG_ERR_ARG,
               "small_dgemm_diag_batch: too many blocks");
  if (count == 0) return;
  SgBatch b{};
  int dmax = 0;
  for (int i = 0; i < count; ++i) {
    LOBPCG_CHECK(dim[i] >= 1 && dim[i] <= kSmallGemmMax && off[i] >= 0, LOBPCG_ERR_ARG,
                 "small_dgemm_diag_batch: bad block");
    b.off[i] = off[i];
    b.dim[i] = dim[i];
    dmax = dim[i] > dmax ? dim[i] : dmax;
  }
  launch<false, false>(dmax, dmax, dmax, 1.0, A, lda, B, ldb, 0.0, C, ldc, b, count, s);
}

}  // namespace lobpcg
