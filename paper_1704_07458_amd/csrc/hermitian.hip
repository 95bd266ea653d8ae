// Complex Hermitian pencils through the real embedding (see hermitian.hpp).
#include "hermitian.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "kernels.hpp"

namespace lobpcg {

#define LOBPCG_ROCBLAS_Z(call)                                                             \
  do {                                                                                     \
    rocblas_status st_ = (call);                                                           \
    if (st_ != rocblas_status_success)                                                     \
      throw ::lobpcg::Error(LOBPCG_ERR_HIP, std::string(#call) + ": " +                    \
                                                rocblas_status_to_string(st_));            \
  } while (0)

namespace {

constexpr int kThreads = 256;

unsigned blocks_for(int64_t total) {
  return (unsigned)std::min<int64_t>((total + kThreads - 1) / kThreads, 65535 * 8);
}

// [X0, i X0] in stacked form: out (2n x 2nx, row-major) =
//   [ re  -im ]
//   [ im   re ]
__global__ void embed_pair_kernel(int64_t n, int nx, const double* __restrict__ re,
                                  const double* __restrict__ im, int64_t ld,
                                  double* __restrict__ out) {
  const int64_t total = n * nx;
  const int64_t ldo = 2 * (int64_t)nx;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / nx;
    const int j = (int)(t % nx);
    const double a = re[r * ld + j], b = im[r * ld + j];
    out[r * ldo + j] = a;
    out[r * ldo + nx + j] = -b;
    out[(n + r) * ldo + j] = b;
    out[(n + r) * ldo + nx + j] = a;
  }
}

// Z(:, j) = sign * (Y(1:n, j) + i Y(n+1:2n, j)); Y row-major 2n x m, Z column-major n x m.
__global__ void stack_to_complex_kernel(int64_t n, int m, const double* __restrict__ Y,
                                        int64_t ldy, double2* __restrict__ Z, double sign) {
  const int64_t total = n * m;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / m;
    const int j = (int)(t % m);
    Z[(int64_t)j * n + r] = make_double2(sign * Y[r * ldy + j], sign * Y[(n + r) * ldy + j]);
  }
}

__global__ void complex_to_stack_kernel(int64_t n, int m, const double2* __restrict__ Z,
                                        double* __restrict__ Y, int64_t ldy) {
  const int64_t total = n * m;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / m;
    const int j = (int)(t % m);
    const double2 z = Z[(int64_t)j * n + r];
    Y[r * ldy + j] = z.x;
    Y[(n + r) * ldy + j] = z.y;
  }
}

// V(:, j) /= sqrt(mu[j]) (mu > 0 on the range of Z^H B Z; a non-positive value
// marks a rank deficiency and zeroes the column).
__global__ void scale_cols_kernel(int rows, int cols, double2* __restrict__ V, int64_t ld,
                                  const double* __restrict__ mu) {
  const int64_t total = (int64_t)rows * cols;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / rows);
    const int i = (int)(t % rows);
    const double m = mu[j];
    const double s = m > 0.0 ? 1.0 / sqrt(m) : 0.0;
    double2 v = V[(int64_t)j * ld + i];
    V[(int64_t)j * ld + i] = make_double2(v.x * s, v.y * s);
  }
}

// Descending order for the largest pairs: theta and the columns of U reversed.
__global__ void reverse_kernel(int k, double* __restrict__ theta, double2* __restrict__ U,
                               int64_t ld) {
  const int64_t total = (int64_t)(k / 2) * (k + 1);
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int j = (int)(t / (k + 1));
    const int i = (int)(t % (k + 1));
    const int jj = k - 1 - j;
    if (i == k) {
      const double a = theta[j];
      theta[j] = theta[jj];
      theta[jj] = a;
    } else {
      const double2 a = U[(int64_t)j * ld + i];
      U[(int64_t)j * ld + i] = U[(int64_t)jj * ld + i];
      U[(int64_t)jj * ld + i] = a;
    }
  }
}

// Criterion (9) of complex pair j: ||A x - theta B x|| / ((||A|| + |theta| ||B||) ||x||).
// One workgroup per column, fixed-order sums.
__global__ __launch_bounds__(kThreads) void rho_kernel(int64_t n, const double2* __restrict__ AX,
                                                       const double2* __restrict__ BX,
                                                       const double2* __restrict__ X,
                                                       const double* __restrict__ theta,
                                                       double normA, double normB,
                                                       double* __restrict__ rho) {
  __shared__ double sr[kThreads], sx[kThreads];
  const int j = blockIdx.x;
  const double th = theta[j];
  double ar = 0.0, ax = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += kThreads) {
    const double2 a = AX[(int64_t)j * n + r], b = BX[(int64_t)j * n + r];
    const double2 x = X[(int64_t)j * n + r];
    const double re = a.x - th * b.x, im = a.y - th * b.y;
    ar = fma(re, re, fma(im, im, ar));
    ax = fma(x.x, x.x, fma(x.y, x.y, ax));
  }
  sr[threadIdx.x] = ar;
  sx[threadIdx.x] = ax;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      sr[threadIdx.x] += sr[threadIdx.x + s];
      sx[threadIdx.x] += sx[threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) rho[j] = sqrt(sr[0]) / ((normA + fabs(th) * normB) * sqrt(sx[0]));
}

// X (column-major n x count, complex) -> Xre, Xim (row-major n x count, ldx).
__global__ void split_out_kernel(int64_t n, int count, const double2* __restrict__ X,
                                 double* __restrict__ Xre, double* __restrict__ Xim,
                                 int64_t ldx) {
  const int64_t total = n * count;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = t / count;
    const int j = (int)(t % count);
    const double2 z = X[(int64_t)j * n + r];
    if (Xre) Xre[r * ldx + j] = z.x;
    if (Xim) Xim[r * ldx + j] = z.y;
  }
}

// Host copy of a complex CSR (device input copied back first).
struct HostZcsr {
  std::vector<int64_t> rowptr;
  std::vector<int32_t> colind;
  std::vector<double> re, im;
};

HostZcsr to_host(const lobpcg_zcsr* M) {
  LOBPCG_CHECK(M->n > 0 && M->nnz >= 0, LOBPCG_ERR_ARG, "complex CSR: bad n or nnz");
  LOBPCG_CHECK(M->n < (int64_t{1} << 30), LOBPCG_ERR_ARG,
               "complex CSR: n too large for the order-2n embedding's int32 columns");
  LOBPCG_CHECK(M->rowptr && (M->nnz == 0 || (M->colind && M->values_re && M->values_im)),
               LOBPCG_ERR_ARG, "complex CSR: NULL array");
  HostZcsr h;
  h.rowptr.resize(M->n + 1);
  h.colind.resize(M->nnz);
  h.re.resize(M->nnz);
  h.im.resize(M->nnz);
  auto get = [&](void* dst, const void* src, size_t bytes) {
    if (M->on_device) LOBPCG_HIP(hipMemcpy(dst, src, bytes, hipMemcpyDeviceToHost));
    else std::memcpy(dst, src, bytes);
  };
  get(h.rowptr.data(), M->rowptr, sizeof(int64_t) * (M->n + 1));
  if (M->nnz) {
    get(h.colind.data(), M->colind, sizeof(int32_t) * M->nnz);
    get(h.re.data(), M->values_re, sizeof(double) * M->nnz);
    get(h.im.data(), M->values_im, sizeof(double) * M->nnz);
  }
  LOBPCG_CHECK(h.rowptr[0] == 0 && h.rowptr[M->n] == M->nnz, LOBPCG_ERR_ARG,
               "complex CSR: rowptr[0] != 0 or rowptr[n] != nnz");
  for (int64_t r = 0; r < M->n; ++r)
    LOBPCG_CHECK(h.rowptr[r] <= h.rowptr[r + 1], LOBPCG_ERR_ARG,
                 "complex CSR: decreasing row pointers");
  return h;
}

// The real embedding [Re, -Im; Im, Re] of order 2n in CSR (sorted columns:
// row r lists the columns c of row r, then n + c).
struct Embedded {
  std::vector<int64_t> rowptr;
  std::vector<int32_t> colind;
  std::vector<double> values;
  lobpcg_csr csr{};
};

void embed(const HostZcsr& h, int64_t n, Embedded& e) {
  const int64_t nnz = (int64_t)h.colind.size();
  e.rowptr.resize(2 * n + 1);
  e.colind.resize(4 * nnz);
  e.values.resize(4 * nnz);
  int64_t q = 0;
  e.rowptr[0] = 0;
  for (int half = 0; half < 2; ++half) {
    for (int64_t r = 0; r < n; ++r) {
      for (int64_t p = h.rowptr[r]; p < h.rowptr[r + 1]; ++p) {
        e.colind[q] = h.colind[p];
        e.values[q++] = half == 0 ? h.re[p] : h.im[p];
      }
      for (int64_t p = h.rowptr[r]; p < h.rowptr[r + 1]; ++p) {
        e.colind[q] = (int32_t)(n + h.colind[p]);
        e.values[q++] = half == 0 ? -h.im[p] : h.re[p];
      }
      e.rowptr[half * n + r + 1] = q;
    }
  }
  e.csr.n = 2 * n;
  e.csr.nnz = 4 * nnz;
  e.csr.rowptr = e.rowptr.data();
  e.csr.colind = e.colind.data();
  e.csr.values = e.values.data();
  e.csr.on_device = 0;
}

}  // namespace

Hermitian::Hermitian(const lobpcg_zcsr* A, const lobpcg_zcsr* B, int k,
                     const lobpcg_options& opt) {
  LOBPCG_CHECK(A != nullptr, LOBPCG_ERR_ARG, "A is NULL");
  LOBPCG_CHECK(k >= 1, LOBPCG_ERR_ARG, "k must be >= 1");
  LOBPCG_CHECK(!B || B->n == A->n, LOBPCG_ERR_ARG, "B must have the order of A");
  n_ = A->n;
  k_ = k;
  nx_ = opt.block_size > 0 ? opt.block_size : k + (k + 9) / 10;
  LOBPCG_CHECK(nx_ >= k, LOBPCG_ERR_ARG, "block_size must be >= k");
  seed_ = opt.seed;
  Embedded ea, eb;
  embed(to_host(A), n_, ea);
  if (B) embed(to_host(B), n_, eb);
  lobpcg_options o = opt;
  o.block_size = 2 * nx_;
  solver_.reset(new Solver(&ea.csr, B ? &eb.csr : nullptr, 2 * k, o));
  AllocatorScope scope(solver_->allocator());
  LOBPCG_ROCBLAS_Z(rocblas_create_handle(&h_));
  LOBPCG_ROCBLAS_Z(rocblas_set_stream(h_, solver_->stream()));
  LOBPCG_ROCBLAS_Z(rocblas_set_atomics_mode(h_, rocblas_atomics_not_allowed));
  const int k2 = 2 * k_;
  const size_t cz = sizeof(double2);
  Xr_.alloc(sizeof(double) * 2 * n_ * std::max(k2, 2 * nx_));
  Y_.alloc(sizeof(double) * 2 * n_ * std::max(k2, 2 * nx_));
  Z_.alloc(cz * n_ * k2);
  if (solver_->has_B()) {
    BZ_.alloc(cz * n_ * k2);
    BQ_.alloc(cz * n_ * k_);
  }
  Q_.alloc(cz * n_ * k_);
  AQ_.alloc(cz * n_ * k_);
  M_.alloc(cz * (size_t)k2 * k2);
  V_.alloc(cz * n_ * k_);
  mu_.alloc(sizeof(double) * k2);
  e_.alloc(sizeof(double) * k2);
  theta_.alloc(sizeof(double) * k_);
  rho_.alloc(sizeof(double) * k_);
  info_.alloc(sizeof(int32_t) * 2);
  library_workspace();
}

Hermitian::~Hermitian() {
  if (solver_) (void)hipStreamSynchronize(solver_->stream());
  if (h_) rocblas_destroy_handle(h_);
}

// Device workspace of the complex library calls at their sizes (size query,
// nothing computed), from the handle's allocator.
void Hermitian::library_workspace() {
  const int k2 = 2 * k_;
  auto* M = M_.as<rocblas_double_complex>();
  auto* Z = Z_.as<rocblas_double_complex>();
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  size_t bytes = 0;
  LOBPCG_ROCBLAS_Z(rocblas_start_device_memory_size_query(h_));
  (void)rocsolver_zheevd(h_, rocblas_evect_original, rocblas_fill_upper, k2, M, k2,
                         mu_.as<double>(), e_.as<double>(), info_.as<rocblas_int>());
  (void)rocblas_zgemm(h_, rocblas_operation_conjugate_transpose, rocblas_operation_none, k2, k2,
                      (rocblas_int)n_, &one, Z, (rocblas_int)n_, Z, (rocblas_int)n_, &zero, M, k2);
  (void)rocblas_zgemm(h_, rocblas_operation_none, rocblas_operation_none, (rocblas_int)n_, k_, k2,
                      &one, Z, (rocblas_int)n_, M, k2, &zero, Q_.as<rocblas_double_complex>(),
                      (rocblas_int)n_);
  LOBPCG_ROCBLAS_Z(rocblas_stop_device_memory_size_query(h_, &bytes));
  lib_ws_.alloc(std::max<size_t>(bytes, 256));
  LOBPCG_ROCBLAS_Z(rocblas_set_workspace(h_, lib_ws_.get(), lib_ws_.size()));
}

int Hermitian::solve(double tol, const double* X0re, const double* X0im, bool x0_dev,
                     lobpcg_precond_fn K, void* Kuser, lobpcg_info* info) {
  LOBPCG_CHECK((X0re == nullptr) == (X0im == nullptr), LOBPCG_ERR_ARG,
               "give both parts of X0 or neither");
  AllocatorScope scope(solver_->allocator());
  const hipStream_t s = solver_->stream();
  const int64_t blk = n_ * nx_;
  double* re = Y_.as<double>();
  double* im = re + blk;
  if (X0re == nullptr) {
    // the seeded 2n x n_x Gaussian block: real parts on top, imaginary below
    launch_gaussian(2 * n_, nx_, re, nx_, seed_, kStreamInitialBlock, s);
  } else {
    const hipMemcpyKind kind = x0_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    LOBPCG_HIP(hipMemcpyAsync(re, X0re, sizeof(double) * blk, kind, s));
    LOBPCG_HIP(hipMemcpyAsync(im, X0im, sizeof(double) * blk, kind, s));
  }
  double* X0 = Xr_.as<double>();  // 2n x 2n_x paired block (the solve copies it)
  hipLaunchKernelGGL(embed_pair_kernel, dim3(blocks_for(blk)), dim3(kThreads), 0, s, n_, nx_, re,
                     im, (int64_t)nx_, X0);
  LOBPCG_HIP(hipGetLastError());
  extracted_ = false;
  return solver_->solve(tol, X0, true, K, Kuser, info);
}

void Hermitian::extract() {
  AllocatorScope scope(solver_->allocator());
  const hipStream_t s = solver_->stream();
  const int k2 = 2 * k_;
  const bool haveB = solver_->has_B();
  const rocblas_double_complex one(1.0, 0.0), zero(0.0, 0.0);
  auto zc = [](DevBuf& b) { return b.as<rocblas_double_complex>(); };
  // 1. the 2k leading real Ritz vectors and their complex forms z_j
  LOBPCG_CHECK(solver_->eigpairs(k2, nullptr, Xr_.as<double>(), k2, nullptr, true) == LOBPCG_OK,
               LOBPCG_ERR_HIP, "eigpairs of the embedding failed");
  const unsigned gz = blocks_for(n_ * k2);
  hipLaunchKernelGGL(stack_to_complex_kernel, dim3(gz), dim3(kThreads), 0, s, n_, k2,
                     Xr_.as<double>(), (int64_t)k2, Z_.as<double2>(), 1.0);
  rocblas_double_complex* BZ = zc(Z_);
  if (haveB) {
    solver_->apply(true, Xr_.as<double>(), k2, Y_.as<double>(), k2, k2);
    hipLaunchKernelGGL(stack_to_complex_kernel, dim3(gz), dim3(kThreads), 0, s, n_, k2,
                       Y_.as<double>(), (int64_t)k2, BZ_.as<double2>(), 1.0);
    BZ = zc(BZ_);
  }
  LOBPCG_HIP(hipGetLastError());
  // 2. M = Z^H B Z (rank k); its k leading eigenvectors V (eigenvalues mu)
  //    give the B-orthonormal basis Q = Z V mu^-1/2 of the complex span
  LOBPCG_ROCBLAS_Z(rocblas_zgemm(h_, rocblas_operation_conjugate_transpose,
                                 rocblas_operation_none, k2, k2, (rocblas_int)n_, &one, zc(Z_),
                                 (rocblas_int)n_, BZ, (rocblas_int)n_, &zero, zc(M_), k2));
  LOBPCG_ROCBLAS_Z(rocsolver_zheevd(h_, rocblas_evect_original, rocblas_fill_upper, k2, zc(M_),
                                    k2, mu_.as<double>(), e_.as<double>(),
                                    info_.as<rocblas_int>()));
  rocblas_double_complex* Vk = zc(M_) + (size_t)k_ * k2;
  hipLaunchKernelGGL(scale_cols_kernel, dim3(blocks_for((int64_t)k2 * k_)), dim3(kThreads), 0, s,
                     k2, k_, reinterpret_cast<double2*>(Vk), (int64_t)k2, mu_.as<double>() + k_);
  LOBPCG_HIP(hipGetLastError());
  LOBPCG_ROCBLAS_Z(rocblas_zgemm(h_, rocblas_operation_none, rocblas_operation_none,
                                 (rocblas_int)n_, k_, k2, &one, zc(Z_), (rocblas_int)n_, Vk, k2,
                                 &zero, zc(Q_), (rocblas_int)n_));
  rocblas_double_complex* BQ = zc(Q_);
  if (haveB) {
    LOBPCG_ROCBLAS_Z(rocblas_zgemm(h_, rocblas_operation_none, rocblas_operation_none,
                                   (rocblas_int)n_, k_, k2, &one, BZ, (rocblas_int)n_, Vk, k2,
                                   &zero, zc(BQ_), (rocblas_int)n_));
    BQ = zc(BQ_);
  }
  // 3. A Q with the stored embedding (negated in the largest mode)
  const unsigned gq = blocks_for(n_ * k_);
  hipLaunchKernelGGL(complex_to_stack_kernel, dim3(gq), dim3(kThreads), 0, s, n_, k_,
                     Q_.as<double2>(), Y_.as<double>(), (int64_t)k_);
  LOBPCG_HIP(hipGetLastError());
  solver_->apply(false, Y_.as<double>(), k_, Xr_.as<double>(), k_, k_);
  hipLaunchKernelGGL(stack_to_complex_kernel, dim3(gq), dim3(kThreads), 0, s, n_, k_,
                     Xr_.as<double>(), (int64_t)k_, AQ_.as<double2>(),
                     solver_->largest() ? -1.0 : 1.0);
  LOBPCG_HIP(hipGetLastError());
  // 4. complex Rayleigh-Ritz: H = Q^H A Q = U Theta U^H, X = Q U
  rocblas_double_complex* H = zc(M_);  // M and V are no longer needed
  LOBPCG_ROCBLAS_Z(rocblas_zgemm(h_, rocblas_operation_conjugate_transpose,
                                 rocblas_operation_none, k_, k_, (rocblas_int)n_, &one, zc(Q_),
                                 (rocblas_int)n_, zc(AQ_), (rocblas_int)n_, &zero, H, k_));
  LOBPCG_ROCBLAS_Z(rocsolver_zheevd(h_, rocblas_evect_original, rocblas_fill_upper, k_, H, k_,
                                    theta_.as<double>(), e_.as<double>(),
                                    info_.as<rocblas_int>() + 1));
  if (solver_->largest()) {
    hipLaunchKernelGGL(reverse_kernel, dim3(blocks_for((int64_t)(k_ / 2) * (k_ + 1) + 1)),
                       dim3(kThreads), 0, s, k_, theta_.as<double>(),
                       reinterpret_cast<double2*>(H), (int64_t)k_);
    LOBPCG_HIP(hipGetLastError());
  }
  // X = Q U (into V_), A X = (A Q) U (into Z_), B X = (B Q) U (into the first
  // n k entries of BZ_, or X itself when B = I)
  auto* X = zc(V_);
  LOBPCG_ROCBLAS_Z(rocblas_zgemm(h_, rocblas_operation_none, rocblas_operation_none,
                                 (rocblas_int)n_, k_, k_, &one, zc(Q_), (rocblas_int)n_, H, k_,
                                 &zero, X, (rocblas_int)n_));
  auto* AX = zc(Z_);
  LOBPCG_ROCBLAS_Z(rocblas_zgemm(h_, rocblas_operation_none, rocblas_operation_none,
                                 (rocblas_int)n_, k_, k_, &one, zc(AQ_), (rocblas_int)n_, H, k_,
                                 &zero, AX, (rocblas_int)n_));
  rocblas_double_complex* BX = X;
  if (haveB) {
    BX = zc(BZ_);
    LOBPCG_ROCBLAS_Z(rocblas_zgemm(h_, rocblas_operation_none, rocblas_operation_none,
                                   (rocblas_int)n_, k_, k_, &one, BQ, (rocblas_int)n_, H, k_,
                                   &zero, BX, (rocblas_int)n_));
  }
  // 5. criterion (9) of each complex pair with the sketch norms
  hipLaunchKernelGGL(rho_kernel, dim3(k_), dim3(kThreads), 0, s, n_,
                     reinterpret_cast<const double2*>(AX), reinterpret_cast<const double2*>(BX),
                     reinterpret_cast<const double2*>(X), theta_.as<double>(),
                     solver_->norm_A_est(), solver_->norm_B_est(), rho_.as<double>());
  LOBPCG_HIP(hipGetLastError());
  int32_t hinfo[2] = {0, 0};
  LOBPCG_HIP(hipMemcpyAsync(hinfo, info_.get(), sizeof(hinfo), hipMemcpyDeviceToHost, s));
  LOBPCG_HIP(hipStreamSynchronize(s));
  LOBPCG_CHECK(hinfo[0] == 0 && hinfo[1] == 0, LOBPCG_ERR_BREAKDOWN,
               "complex extraction: Hermitian eigensolver did not converge");
  extracted_ = true;
}

int Hermitian::eigpairs(int count, double* lambda, double* Xre, double* Xim, int64_t ldx,
                        double* rho, bool on_device) {
  LOBPCG_CHECK(solver_->solved(), LOBPCG_ERR_STATE, "eigpairs called before a successful solve");
  LOBPCG_CHECK(count >= 0 && count <= k_, LOBPCG_ERR_ARG, "count must be in [0, k]");
  if (count == 0) return LOBPCG_OK;
  if (!extracted_) extract();
  AllocatorScope scope(solver_->allocator());
  const hipStream_t s = solver_->stream();
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (lambda) LOBPCG_HIP(hipMemcpyAsync(lambda, theta_.get(), sizeof(double) * count, kind, s));
  if (rho) LOBPCG_HIP(hipMemcpyAsync(rho, rho_.get(), sizeof(double) * count, kind, s));
  if (Xre || Xim) {
    LOBPCG_CHECK(ldx >= count, LOBPCG_ERR_ARG, "ldx < count");
    const unsigned g = blocks_for(n_ * count);
    if (on_device) {
      hipLaunchKernelGGL(split_out_kernel, dim3(g), dim3(kThreads), 0, s, n_, count,
                         V_.as<double2>(), Xre, Xim, ldx);
      LOBPCG_HIP(hipGetLastError());
    } else {
      double* sre = Y_.as<double>();
      double* sim = sre + n_ * count;
      hipLaunchKernelGGL(split_out_kernel, dim3(g), dim3(kThreads), 0, s, n_, count,
                         V_.as<double2>(), sre, sim, (int64_t)count);
      LOBPCG_HIP(hipGetLastError());
      if (Xre)
        LOBPCG_HIP(hipMemcpy2DAsync(Xre, sizeof(double) * ldx, sre, sizeof(double) * count,
                                    sizeof(double) * count, n_, hipMemcpyDeviceToHost, s));
      if (Xim)
        LOBPCG_HIP(hipMemcpy2DAsync(Xim, sizeof(double) * ldx, sim, sizeof(double) * count,
                                    sizeof(double) * count, n_, hipMemcpyDeviceToHost, s));
    }
  }
  LOBPCG_HIP(hipStreamSynchronize(s));
  return LOBPCG_OK;
}

}  // namespace lobpcg
