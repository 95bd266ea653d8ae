// Gradient of a loss on computed eigenpairs with respect to the stored values
// of A (and of B for a generalised pencil), from first-order perturbation
// theory of A x = lambda B x with X^T B X = I:
//   d lambda_i = x_i^T (dA - lambda_i dB) x_i,
//   y_i = -sum_{j != i} x_j (x_j^T xbar_i) / (lambda_j - lambda_i),
//   gradA_rc = sum_i lambda_bar_i x_i(r) x_i(c) + 1/2 sum_i (y_i(r) x_i(c) + x_i(r) y_i(c)),
//   gradB_rc = sum_i a_i x_i(r) x_i(c) + 1/2 sum_i b_i (y_i(r) x_i(c) + x_i(r) y_i(c)),
//   a_i = -(lambda_bar_i lambda_i + 1/2 xbar_i^T x_i), b_i = -lambda_i
// (the 1/2 xbar_i^T x_i term comes from keeping x_i^T B x_i = 1).
// y_i is split into the part inside the computed block X (a count x count sum)
// and the part outside, which solves the projected shifted system
//   Pi^T (A - lambda_i B) Pi z_i = -Pi^T xbar_i,  y_i = Pi z_i,  Pi = I - X X^T B
// (Pi = I - X X^T when B = I) by conjugate gradients run on all columns at once
// (one sparse product with A, and one with B, per step for the whole block).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "kernels.hpp"
#include "solver.hpp"

namespace lobpcg {
namespace {

constexpr int kWave = 64;

// coef(j, i) = -G(j, i) / (lambda_j - lambda_i), j != i (column-major count x count).
__global__ void inblock_coef_kernel(int m, const double* __restrict__ G, int64_t ldg,
                                    const double* __restrict__ lam, double* __restrict__ coef,
                                    int64_t ldc) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= m * m) return;
  const int j = idx % m, i = idx / m;
  coef[j + (int64_t)i * ldc] = (j == i) ? 0.0 : -G[j + (int64_t)i * ldg] / (lam[j] - lam[i]);
}

// Y = s * X (n x m row-major blocks).
__global__ void scale_copy_kernel(int64_t n, int m, double s, const double* __restrict__ X,
                                  int64_t ldx, double* __restrict__ Y, int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t r = idx / m;
  const int c = (int)(idx % m);
  Y[r * ldy + c] = s * X[r * ldx + c];
}

// AP(:, i) -= lam_i P(:, i)
__global__ void shift_kernel(int64_t n, int m, const double* __restrict__ lam,
                             const double* __restrict__ P, int64_t ldp, double* __restrict__ AP,
                             int64_t ldap) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t r = idx / m;
  const int c = (int)(idx % m);
  AP[r * ldap + c] -= lam[c] * P[r * ldp + c];
}

// Per-column dot products of two blocks, partial sums per row block.
constexpr int kRows = 256;
__global__ __launch_bounds__(256) void coldot_kernel(int64_t n, int m, const double* __restrict__ A,
                                                     int64_t lda, const double* __restrict__ B,
                                                     int64_t ldb, double* __restrict__ part) {
  __shared__ double sq[4][kWave];
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  const int j = blockIdx.y * kWave + lane;
  const int64_t r0 = (int64_t)blockIdx.x * kRows;
  const int64_t r1 = std::min<int64_t>(n, r0 + kRows);
  double acc = 0.0;
  if (j < m)
    for (int64_t r = r0 + wave; r < r1; r += 4) acc = fma(A[r * lda + j], B[r * ldb + j], acc);
  sq[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && j < m)
    part[(int64_t)blockIdx.x * m + j] = ((sq[0][lane] + sq[1][lane]) + sq[2][lane]) + sq[3][lane];
}

__global__ void colsum_finish_kernel(int m, int nb, const double* __restrict__ part,
                                     double* __restrict__ out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double a = 0.0;
  for (int t = 0; t < nb; ++t) a += part[(int64_t)t * m + j];
  out[j] = a;
}

// alpha_i = rr_i / pAp_i for active columns.  A column whose curvature pAp is
// not positive (or not finite) has reached the rounding floor of the projected
// operator, which is positive definite in exact arithmetic: it stops there
// (alpha = 0, inactive) and is counted in *nbreak.
__global__ void cg_alpha_kernel(int m, const double* rr, const double* pap, int* active,
                                double* alpha, int* nbreak) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double a = 0.0;
  if (active[j]) {
    if (pap[j] > 0.0 && pap[j] < INFINITY) {
      a = rr[j] / pap[j];
    } else {
      active[j] = 0;
      atomicAdd(nbreak, 1);
    }
  }
  alpha[j] = a;
}

// Z += alpha P; R -= alpha AP
__global__ void cg_step_kernel(int64_t n, int m, const double* __restrict__ alpha,
                               const double* __restrict__ P, const double* __restrict__ AP,
                               double* __restrict__ Z, double* __restrict__ R, int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t r = idx / m;
  const int c = (int)(idx % m);
  const double a = alpha[c];
  Z[r * ld + c] += a * P[r * ld + c];
  R[r * ld + c] -= a * AP[r * ld + c];
}

// beta_i = rr_new_i / rr_i; update active flags; rr = rr_new; count active.
__global__ __launch_bounds__(256) void cg_beta_kernel(int m, double* rr, const double* rr_new,
                                                      const double* bn2, double tol2, int* active,
                                                      double* beta, int* nactive) {
  __shared__ int s[256];
  int cnt = 0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const bool was = active[j] != 0;
    const bool still = was && rr_new[j] > tol2 * bn2[j];
    beta[j] = still && rr[j] > 0.0 ? rr_new[j] / rr[j] : 0.0;
    if (was) rr[j] = rr_new[j];
    active[j] = still ? 1 : 0;
    cnt += still ? 1 : 0;
  }
  s[threadIdx.x] = cnt;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *nactive = s[0];
}

// P = R + beta P (columns with beta = 0 and inactive keep P = R, harmless: alpha = 0).
__global__ void cg_dir_kernel(int64_t n, int m, const double* __restrict__ beta,
                              const double* __restrict__ R, double* __restrict__ P, int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t r = idx / m;
  const int c = (int)(idx % m);
  P[r * ld + c] = R[r * ld + c] + beta[c] * P[r * ld + c];
}

// Y += X (n x m row-major blocks).
__global__ void axpy_kernel(int64_t n, int m, const double* __restrict__ X, int64_t ldx,
                            double* __restrict__ Y, int64_t ldy) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * m) return;
  const int64_t r = idx / m;
  const int c = (int)(idx % m);
  Y[r * ldy + c] += X[r * ldx + c];
}

__global__ void init_active_kernel(int m, const double* bn2, int* active) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < m) active[j] = bn2[j] > 0.0 ? 1 : 0;
}

// One wave per row; lanes over eigenpair index i (chunks of 64), shuffle sums.
// grad[p] = sum_i a_i x_i(r) x_i(c) + 1/2 b_i (y_i(r) x_i(c) + x_i(r) y_i(c)); b = NULL means 1.
__global__ __launch_bounds__(256) void scatter_grad_kernel(
    int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind, int m,
    const double* __restrict__ X, int64_t ldx, const double* __restrict__ Y, int64_t ldy,
    const double* __restrict__ lbar, const double* __restrict__ ycoef,
    double* __restrict__ grad) {
  const int64_t r = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (r >= n) return;
  for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
    const int64_t c = colind[p];
    double acc = 0.0;
    for (int i0 = 0; i0 < m; i0 += kWave) {
      const int i = i0 + lane;
      if (i < m) {
        const double xr = X[r * ldx + i], xc = X[c * ldx + i];
        const double yr = Y[r * ldy + i], yc = Y[c * ldy + i];
        acc += lbar[i] * xr * xc + 0.5 * (ycoef ? ycoef[i] : 1.0) * (yr * xc + xr * yc);
      }
    }
    for (int off = kWave / 2; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if (lane == 0) grad[p] = acc;
  }
}

// a_i = -(lambda_bar_i lambda_i + 1/2 xbar_i^T x_i), b_i = -lambda_i, with
// xbar_i^T x_i = G(i, i) of G = X^T Xbar (column-major, ldg; NULL = 0).
__global__ void b_coef_kernel(int m, const double* __restrict__ lbar,
                              const double* __restrict__ lam, const double* __restrict__ G,
                              int64_t ldg, double* __restrict__ a, double* __restrict__ b) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const double xx = G ? G[i + (int64_t)i * ldg] : 0.0;
  a[i] = -(lbar[i] * lam[i] + 0.5 * xx);
  b[i] = -lam[i];
}

inline unsigned nblk(int64_t total) { return (unsigned)((total + 255) / 256); }

}  // namespace

int Solver::adjoint(int count, const double* lambda_bar, const double* X_bar, int64_t ld_xbar,
                    double* grad, double* grad_B, double cg_tol, int cg_maxit,
                    int32_t* cg_iters) {
  LOBPCG_CHECK(solved_, LOBPCG_ERR_STATE, "adjoint called before a solve");
  LOBPCG_CHECK(opt_.largest == 0, LOBPCG_ERR_ARG,
               "adjoint is not provided for the largest-eigenpair mode");
  LOBPCG_CHECK(count >= 1 && count <= nx_, LOBPCG_ERR_ARG, "count must be in [1, n_x]");
  LOBPCG_CHECK(grad != nullptr, LOBPCG_ERR_ARG, "grad is NULL");
  LOBPCG_CHECK(grad_B == nullptr || haveB_, LOBPCG_ERR_ARG, "grad_B given but B = I");
  LOBPCG_CHECK(X_bar == nullptr || ld_xbar >= count, LOBPCG_ERR_ARG, "ld_xbar < count");
  AllocatorScope scope(&alloc_);
  const double tol = cg_tol > 0 ? cg_tol : 1e-12;
  const int maxit = cg_maxit > 0 ? cg_maxit : 10000;
  const int64_t n = n_;
  const int m = count;
  const int64_t ld = round_up(m, 16);
  const double* X = Xres_;
  const int64_t ldx = ldS_;
  const double* lam = theta_.as<double>();
  hipStream_t s = s_;
  const bool gen = haveB_;

  DevBuf Y(sizeof(double) * n * ld), Z(sizeof(double) * n * ld), R(sizeof(double) * n * ld),
      P(sizeof(double) * n * ld), AP(sizeof(double) * n * ld);
  // B != I: B X, B P (then B Pi P) and Pi P
  DevBuf BXb, BPb, Qb;
  if (gen) {
    BXb.alloc(sizeof(double) * n * ld);
    BPb.alloc(sizeof(double) * n * ld);
    Qb.alloc(sizeof(double) * n * ld);
  }
  const int64_t nb = (n + kRows - 1) / kRows;
  DevBuf small(sizeof(double) * (size_t)(m * m * 3 + 16 * m + 16));
  DevBuf part(sizeof(double) * (size_t)std::max<int64_t>(nb * m, 1));
  DevBuf gws(gram_workspace_bound(n, m, m, false));
  DevBuf flags(sizeof(int) * (m + 4));
  double* G = small.as<double>();
  double* G0 = G + m * m;    // X^T Xbar, kept for the B coefficients
  double* vec = G0 + m * m;
  double* lb = vec;          // m
  double* rr = lb + m;       // m
  double* rrn = rr + m;      // m
  double* pap = rrn + m;     // m
  double* alpha = pap + m;   // m
  double* beta = alpha + m;  // m
  double* bn2 = beta + m;    // m
  double* coefA = bn2 + m;   // m  (a_i of the B gradient)
  double* coefB = coefA + m; // m  (b_i of the B gradient)
  double* coef = coefB + m;  // m x m (in-block coefficients) -- fits: 3 m^2 + 16 m + 16
  int* active = flags.as<int>();
  int* nact = active + m;

  std::vector<double> hlb(m, 0.0);
  if (lambda_bar) std::copy(lambda_bar, lambda_bar + m, hlb.begin());
  LOBPCG_HIP(hipMemcpyAsync(lb, hlb.data(), sizeof(double) * m, hipMemcpyHostToDevice, s));

  double* Yp = Y.as<double>();
  double* Zp = Z.as<double>();
  double* Rp = R.as<double>();
  double* Pp = P.as<double>();
  double* APp = AP.as<double>();
  double* BX = gen ? BXb.as<double>() : nullptr;
  double* BPp = gen ? BPb.as<double>() : nullptr;
  double* Qp = gen ? Qb.as<double>() : nullptr;
  // B X (or X itself): Pi^T v = v - BX (X^T v)
  const double* BXe = gen ? BX : X;
  const int64_t ldbx = gen ? ld : ldx;
  const DevCsr* Bm = gen ? &B_ : nullptr;
  auto spmm_dev = [&](const DevCsr& M, const double* in, double* out) {
    launch_spmm<double>(n, M.rowptr.as<int64_t>(), M.colind.as<int32_t>(), M.v64.as<double>(), in,
                        ld, out, ld, m, s);
  };
  auto xt = [&](const double* V, int64_t ldv, double* out) {  // out = X^T V (m x m, cm)
    launch_gram<double>(n, m, m, m, X, ldx, V, ldv, nullptr, 0, out, 0, nullptr, 0, m, 0,
                        gws.get(), s);
  };
  if (gen)
    launch_spmm<double>(n, Bm->rowptr.as<int64_t>(), Bm->colind.as<int32_t>(),
                        Bm->v64.as<double>(), X, ldx, BX, ld, m, s);
  LOBPCG_HIP(hipMemsetAsync(Yp, 0, sizeof(double) * n * ld, s));
  LOBPCG_HIP(hipMemsetAsync(Zp, 0, sizeof(double) * n * ld, s));
  int iters = 0;
  bool converged = true;
  if (X_bar) {
    converged = false;
    // In-block part: Y = X coef, coef(j, i) = -(x_j^T xbar_i) / (lambda_j - lambda_i).
    xt(X_bar, ld_xbar, G0);
    hipLaunchKernelGGL(inblock_coef_kernel, dim3(nblk(m * m)), dim3(256), 0, s, m, G0,
                       (int64_t)m, lam, coef, (int64_t)m);
    launch_update<double>(n, m, m, X, ldx, coef, m, 1.0, 0.0, Yp, ld, s);
    // rhs = -Pi^T xbar = -xbar + BX (X^T xbar)
    hipLaunchKernelGGL(scale_copy_kernel, dim3(nblk(n * m)), dim3(256), 0, s, n, m, -1.0, X_bar,
                       ld_xbar, Rp, ld);
    launch_update<double>(n, m, m, BXe, ldbx, G0, m, 1.0, 1.0, Rp, ld, s);
    // Projected CG, all columns at once.
    launch_copy2d<double, double>(n, m, Rp, ld, Pp, ld, s);
    auto coldot = [&](const double* A1, const double* B1, double* out) {
      hipLaunchKernelGGL(coldot_kernel, dim3((unsigned)nb, (unsigned)((m + 63) / 64)), dim3(256), 0,
                         s, n, m, A1, ld, B1, ld, part.as<double>());
      hipLaunchKernelGGL(colsum_finish_kernel, dim3(nblk(m)), dim3(256), 0, s, m, (int)nb,
                         part.as<double>(), out);
    };
    coldot(Rp, Rp, rr);
    LOBPCG_HIP(hipMemcpyAsync(bn2, rr, sizeof(double) * m, hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(init_active_kernel, dim3(nblk(m)), dim3(256), 0, s, m, bn2, active);
    LOBPCG_HIP(hipMemsetAsync(nact, 0, sizeof(int) * 2, s));
    const double tol2 = tol * tol;
    int32_t* hflag = nullptr;
    LOBPCG_HIP(hipHostMalloc((void**)&hflag, sizeof(int32_t) * 2, hipHostMallocDefault));
    try {
      for (iters = 0; iters < maxit; ++iters) {
        // AP = Pi^T (A - lambda B) Pi P.  B = I: P stays in the range of Pi
        // (the residual is projected every step), so Pi P = P.
        const double* Qs = Pp;
        const double* BQ = Pp;
        if (gen) {
          // Q = Pi P = P - X (X^T B P); B Q = B P - B X (X^T B P)
          spmm_dev(*Bm, Pp, BPp);
          xt(BPp, ld, G);
          launch_copy2d<double, double>(n, m, Pp, ld, Qp, ld, s);
          launch_update<double>(n, m, m, X, ldx, G, m, -1.0, 1.0, Qp, ld, s);
          launch_update<double>(n, m, m, BX, ld, G, m, -1.0, 1.0, BPp, ld, s);
          Qs = Qp;
          BQ = BPp;
        }
        spmm_dev(A_, Qs, APp);
        hipLaunchKernelGGL(shift_kernel, dim3(nblk(n * m)), dim3(256), 0, s, n, m, lam, BQ, ld,
                           APp, ld);
        xt(APp, ld, G);
        launch_update<double>(n, m, m, BXe, ldbx, G, m, -1.0, 1.0, APp, ld, s);
        coldot(Pp, APp, pap);
        hipLaunchKernelGGL(cg_alpha_kernel, dim3(nblk(m)), dim3(256), 0, s, m, rr, pap, active,
                           alpha, nact + 1);
        hipLaunchKernelGGL(cg_step_kernel, dim3(nblk(n * m)), dim3(256), 0, s, n, m, alpha, Pp,
                           APp, Zp, Rp, ld);
        // R <- Pi^T R: AP lies in the range of Pi^T only up to rounding, and the
        // part of R outside it would otherwise accumulate, never decay, and
        // put a floor under ||R|| that the projected operator cannot see.
        xt(Rp, ld, G);
        launch_update<double>(n, m, m, BXe, ldbx, G, m, -1.0, 1.0, Rp, ld, s);
        coldot(Rp, Rp, rrn);
        hipLaunchKernelGGL(cg_beta_kernel, dim3(1), dim3(256), 0, s, m, rr, rrn, bn2, tol2, active,
                           beta, nact);
        hipLaunchKernelGGL(cg_dir_kernel, dim3(nblk(n * m)), dim3(256), 0, s, n, m, beta, Rp, Pp,
                           ld);
        LOBPCG_HIP(hipGetLastError());
        LOBPCG_HIP(hipMemcpyAsync(hflag, nact, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s));
        LOBPCG_HIP(hipStreamSynchronize(s));
        if (hflag[0] == 0) {
          ++iters;
          converged = true;
          break;
        }
      }
    } catch (...) {
      (void)hipHostFree(hflag);
      throw;
    }
    LOBPCG_HIP(hipHostFree(hflag));
    // Z <- Pi Z = Z - X (X^T B Z), then Y += Z (the out-of-block part).
    if (gen) {
      spmm_dev(*Bm, Zp, BPp);
      xt(BPp, ld, G);
    } else {
      xt(Zp, ld, G);
    }
    launch_update<double>(n, m, m, X, ldx, G, m, -1.0, 1.0, Zp, ld, s);
    hipLaunchKernelGGL(axpy_kernel, dim3(nblk(n * m)), dim3(256), 0, s, n, m, Zp, ld, Yp, ld);
  }
  hipLaunchKernelGGL(scatter_grad_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n,
                     A_.rowptr.as<int64_t>(), A_.colind.as<int32_t>(), m, X, ldx, Yp, ld, lb,
                     (const double*)nullptr, grad);
  if (grad_B) {
    hipLaunchKernelGGL(b_coef_kernel, dim3(nblk(m)), dim3(256), 0, s, m, lb, lam,
                       X_bar ? G0 : nullptr, (int64_t)m, coefA, coefB);
    hipLaunchKernelGGL(scatter_grad_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n,
                       B_.rowptr.as<int64_t>(), B_.colind.as<int32_t>(), m, X, ldx, Yp, ld,
                       coefA, coefB, grad_B);
  }
  LOBPCG_HIP(hipGetLastError());
  LOBPCG_HIP(hipStreamSynchronize(s));
  if (cg_iters) *cg_iters = iters;
  return converged ? LOBPCG_OK : LOBPCG_NOT_CONVERGED;
}

}  // namespace lobpcg
