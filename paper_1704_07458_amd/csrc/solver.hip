// Algorithm 8 of arXiv 1704.07458 (robust and efficient LOBPCG) on one GPU.
//
// Storage (row-major, device):
//   S[cur] = [X | P | W]  n x ldS, ping-pong with S[cur^1] for the update
//            [X, P] = S [C_x, C_p] (section 5.1 writes in place through row
//            chunks to save memory; with 288 GB of HBM two copies are cheap and
//            the update needs no chunk buffer).
//   W is stored with reversed column order (section 5.1), so the unconverged
//   columns n_c..n_x-1 of R are the first n_x - n_c columns of the W block.
//   AX, AW (n x ldX): A X is recomputed with the sparse product after every
//   update by default (explicit products), AW for the Gram blocks.
//   BXP = [B X | B P], BW when B != I.
// Projected matrices GA, GB (n_s x n_s, column-major, FP64): the X and P blocks
// come from eqs. (12)-(14) (Theta, 0, Theta_p, I) except in the step after an
// ill-conditioned Cholesky factor; only the W columns are computed (Gram
// kernel), then Algorithm 7 runs on the device in FP64.
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include <rocblas/rocblas.h>

#include "kernels.hpp"

namespace lobpcg {

// Rows per chunk when the Gram blocks go through the library's batched GEMM
// (0: gram_partial_kernel).  Measured on MI355X: for the 64^3 shapes (m x p up
// to 330 x 220) the split-K kernel is faster (46 against 41 TFLOP/s FP64, 82
// against 58 FP32); for the FEM k = 400 and periodic k = 1000 shapes the
// batched GEMM over row chunks runs FP64 at 66-70 TFLOP/s against 43-45, and
// FP32 at 134 against 90 (k = 1000; at k = 400 the two tie in FP32).  FP32
// chunks keep the kernel's bound of 8192 rows per FP32 accumulation.
static int64_t gram_library_rows(bool fp32, int64_t n, int m, int p) {
  const int64_t mp = (int64_t)m * p;
  if (fp32) return mp >= 2000000 ? std::min<int64_t>(n, 8192) : 0;
  if (mp < 500000) return 0;
  return std::min<int64_t>(n, std::max<int64_t>(4096, (n / 32 + 255) / 256 * 256));
}


namespace {
constexpr double kEps64 = 2.220446049250313e-16;
constexpr double kEps32 = 1.1920928955078125e-07;

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

void validate_csr(const lobpcg_csr* M, const char* name, int64_t n_expect,
                  std::vector<int64_t>& rp, std::vector<int32_t>& ci, std::vector<double>& va) {
  LOBPCG_CHECK(M != nullptr, LOBPCG_ERR_ARG, std::string(name) + " is NULL");
  LOBPCG_CHECK(M->n > 0, LOBPCG_ERR_ARG, std::string(name) + ": n must be positive");
  LOBPCG_CHECK(n_expect < 0 || M->n == n_expect, LOBPCG_ERR_ARG,
               std::string(name) + ": dimension mismatch");
  LOBPCG_CHECK(M->rowptr && M->colind && M->values, LOBPCG_ERR_ARG,
               std::string(name) + ": NULL array");
  const int64_t n = M->n;
  rp.resize(n + 1);
  if (M->on_device) {
    LOBPCG_HIP(hipMemcpy(rp.data(), M->rowptr, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost));
  } else {
    std::memcpy(rp.data(), M->rowptr, sizeof(int64_t) * (n + 1));
  }
  LOBPCG_CHECK(rp[0] == 0 && rp[n] == M->nnz, LOBPCG_ERR_ARG,
               std::string(name) + ": rowptr[0] != 0 or rowptr[n] != nnz");
  const int64_t nnz = M->nnz;
  ci.resize(nnz);
  va.resize(nnz);
  if (M->on_device) {
    LOBPCG_HIP(hipMemcpy(ci.data(), M->colind, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
    LOBPCG_HIP(hipMemcpy(va.data(), M->values, sizeof(double) * nnz, hipMemcpyDeviceToHost));
  } else {
    std::memcpy(ci.data(), M->colind, sizeof(int32_t) * nnz);
    std::memcpy(va.data(), M->values, sizeof(double) * nnz);
  }
  for (int64_t r = 0; r < n; ++r) {
    LOBPCG_CHECK(rp[r + 1] >= rp[r], LOBPCG_ERR_ARG,
                 std::string(name) + ": rowptr not monotone at row " + std::to_string(r));
    for (int64_t p = rp[r]; p < rp[r + 1]; ++p) {
      const int32_t c = ci[p];
      LOBPCG_CHECK(c >= 0 && c < n, LOBPCG_ERR_ARG,
                   std::string(name) + ": column index out of range in row " + std::to_string(r));
      LOBPCG_CHECK(p == rp[r] || ci[p - 1] < c, LOBPCG_ERR_ARG,
                   std::string(name) + ": columns not sorted/unique in row " + std::to_string(r));
      LOBPCG_CHECK(std::isfinite(va[p]), LOBPCG_ERR_ARG,
                   std::string(name) + ": non-finite value in row " + std::to_string(r));
    }
  }
}

void upload_csr(DevCsr& D, const std::vector<int64_t>& rp, const std::vector<int32_t>& ci,
                const std::vector<double>& va, bool need32, hipStream_t s) {
  D.n = (int64_t)rp.size() - 1;
  D.nnz = (int64_t)ci.size();
  D.rowptr.alloc(sizeof(int64_t) * rp.size());
  D.colind.alloc(sizeof(int32_t) * std::max<size_t>(ci.size(), 1));
  D.v64.alloc(sizeof(double) * std::max<size_t>(va.size(), 1));
  LOBPCG_HIP(hipMemcpyAsync(D.rowptr.get(), rp.data(), sizeof(int64_t) * rp.size(),
                            hipMemcpyHostToDevice, s));
  if (D.nnz) {
    LOBPCG_HIP(hipMemcpyAsync(D.colind.get(), ci.data(), sizeof(int32_t) * ci.size(),
                              hipMemcpyHostToDevice, s));
    LOBPCG_HIP(hipMemcpyAsync(D.v64.get(), va.data(), sizeof(double) * va.size(),
                              hipMemcpyHostToDevice, s));
  }
  if (need32) {
    D.v32.alloc(sizeof(float) * std::max<size_t>(va.size(), 1));
    launch_copy2d<double, float>(D.nnz, 1, D.v64.as<double>(), 1, D.v32.as<float>(), 1, s);
  }
  LOBPCG_HIP(hipStreamSynchronize(s));  // host vectors go out of scope
}
}  // namespace

template <typename T>
void Blocks<T>::alloc(int64_t n, int64_t ldS, int64_t ldX, bool haveB, bool implicit_products) {
  const size_t e = sizeof(T);
  S[0].alloc(e * n * ldS);
  S[1].alloc(e * n * ldS);
  AX.alloc(e * n * ldX);
  AW.alloc(e * n * ldX);
  U2.alloc(e * n * ldX);
  R.alloc(e * n * ldX);
  if (haveB) {
    BXP.alloc(e * n * 2 * ldX);
    BW.alloc(e * n * ldX);
    MU.alloc(e * n * ldX);
  }
  if (implicit_products) {
    AS[0].alloc(e * n * ldS);
    AS[1].alloc(e * n * ldS);
  }
}

Solver::Solver(const lobpcg_csr* A, const lobpcg_csr* B, int k, const lobpcg_options& opt)
    : opt_(opt) {
  LOBPCG_CHECK((opt.dev_alloc == nullptr) == (opt.dev_free == nullptr), LOBPCG_ERR_ARG,
               "dev_alloc and dev_free must be given together");
  alloc_.alloc = opt.dev_alloc;
  alloc_.free = opt.dev_free;
  alloc_.user = opt.alloc_user;
  AllocatorScope scope(&alloc_);
  s_ = static_cast<hipStream_t>(opt.stream);
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> va;
  validate_csr(A, "A", -1, rp, ci, va);
  n_ = A->n;
  LOBPCG_CHECK(k >= 1, LOBPCG_ERR_ARG, "k must be >= 1");
  k_ = k;
  nx_ = opt.block_size > 0 ? opt.block_size : k + (k + 9) / 10;
  LOBPCG_CHECK(nx_ >= k, LOBPCG_ERR_ARG, "block_size must be >= k");
  LOBPCG_CHECK(3 * (int64_t)nx_ <= n_, LOBPCG_ERR_ARG, "need 3 * block_size <= n");
  LOBPCG_CHECK(opt.implicit_products >= -1 && opt.implicit_products <= 1, LOBPCG_ERR_ARG,
               "implicit_products must be -1, 0 or 1");
  LOBPCG_CHECK(opt.implicit_products != 1 || B == nullptr, LOBPCG_ERR_ARG,
               "implicit product updates need B = I (section 5.2: with B != I the updates "
               "are not safe)");
  LOBPCG_CHECK(opt.ortho_mode == 0 || opt.ortho_mode == 1, LOBPCG_ERR_ARG,
               "ortho_mode must be 0 (orthoDrop) or 1 (ortho)");
  LOBPCG_CHECK(opt.largest == 0 || opt.largest == 1, LOBPCG_ERR_ARG, "largest must be 0/1");
  LOBPCG_CHECK(opt.basic == 0 || opt.basic == 1, LOBPCG_ERR_ARG, "basic must be 0/1");
  // The k largest pairs of (A, B) are the k smallest of (-A, B).
  if (opt.largest)
    for (double& v : va) v = -v;
  LOBPCG_CHECK(opt.precision == 0 || opt.precision == 1, LOBPCG_ERR_ARG, "precision must be 0/1");
  LOBPCG_CHECK(opt.precond >= 0 && opt.precond <= 2, LOBPCG_ERR_ARG, "precond must be 0/1/2");
  const bool split = opt.precision == 1;
  // Validate everything on the host before the first device allocation.
  std::vector<int64_t> brp;
  std::vector<int32_t> bci;
  std::vector<double> bva;
  if (B) validate_csr(B, "B", n_, brp, bci, bva);
  upload_csr(A_, rp, ci, va, split, s_);
  if (B) {
    upload_csr(B_, brp, bci, bva, split, s_);
    haveB_ = true;
  }
  nsmax_ = 3 * nx_;
  ldS_ = round_up(nsmax_, 16);
  ldX_ = round_up(nx_, 16);
  const bool impl = opt.implicit_products == 1;
  b64_.alloc(n_, ldS_, ldX_, haveB_, impl);
  if (split) b32_.alloc(n_, ldS_, ldX_, haveB_, impl);
  const size_t sq = sizeof(double) * (size_t)nsmax_ * nsmax_;
  GA_.alloc(sq);
  GB_.alloc(sq);
  C_.alloc(sizeof(double) * (size_t)nsmax_ * 2 * nx_);
  theta_.alloc(sizeof(double) * nsmax_);
  theta_p_.alloc(sizeof(double) * (size_t)nx_ * nx_);
  rho_.alloc(sizeof(double) * nx_);
  nc_.alloc(sizeof(int32_t) * 4);
  nrm_.alloc(sizeof(double) * (8 * nx_ + 8));
  X0buf_.alloc(sizeof(double) * (size_t)n_ * nx_);
  int64_t ws = gram_workspace_bound(n_, nsmax_, 2 * nx_, split);
  ws = std::max(ws, residual_workspace_bytes(n_, nx_));
  ws = std::max(ws, spmm_residual_workspace_bytes(n_, nx_));
  {
    // partial tiles of the library Gram path at its largest shape (m = n_s,
    // p = 2 n_x); both precisions' chunkings
    const int64_t mp = (int64_t)nsmax_ * 2 * nx_;
    for (int f = 0; f < (split ? 2 : 1); ++f) {
      const int64_t rows = gram_library_rows(f == 1, n_, nsmax_, 2 * nx_);
      if (rows > 0)
        ws = std::max(ws, ((n_ + rows - 1) / rows) * mp * (int64_t)(f == 1 ? 4 : 8));
    }
  }
  ws = std::max(ws, colsq_workspace_bytes(n_, 2 * nx_));
  ws = std::max(ws, jacobi_workspace_bytes(n_));
  work_.alloc(ws);
  if (opt.precond == 1) {
    dinv_.alloc(sizeof(double) * n_);
    launch_jacobi_setup(n_, A_.rowptr.as<int64_t>(), A_.colind.as<int32_t>(), A_.v64.as<double>(),
                        dinv_.as<double>(), work_.get(), s_);
  }
  dense_.reset(new Dense(nsmax_, nx_, s_));
  dense_->set_timer(&timer_);
  {
    // device workspace of the basis-update GEMMs at their largest shape
    rocblas_handle h = dense_->handle();
    size_t bytes = 0;
    LOBPCG_CHECK(rocblas_start_device_memory_size_query(h) == rocblas_status_success,
                 LOBPCG_ERR_HIP, "rocBLAS size query");
    const double one = 1.0, zero = 0.0;
    const float onef = 1.0f, zerof = 0.0f;
    double* Cd = C_.as<double>();
    (void)rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, 2 * nx_,
                        (rocblas_int)n_, nsmax_, &one, Cd, nsmax_, b64_.S[0].as<double>(),
                        (rocblas_int)ldS_, &zero, b64_.S[1].as<double>(), (rocblas_int)ldS_);
    if (split) {
      C32_.alloc(sizeof(float) * (size_t)nsmax_ * 2 * nx_);
      (void)rocblas_sgemm(h, rocblas_operation_transpose, rocblas_operation_none, 2 * nx_,
                          (rocblas_int)n_, nsmax_, &onef, C32_.as<float>(), nsmax_,
                          b32_.S[0].as<float>(), (rocblas_int)ldS_, &zerof,
                          b32_.S[1].as<float>(), (rocblas_int)ldS_);
    }
    // and of the batched Gram GEMMs (R operand n x 2 n_x, L operand n x n_s)
    for (int f = 0; f < (split ? 2 : 1); ++f) {
      const int64_t rows = gram_library_rows(f == 1, n_, nsmax_, 2 * nx_);
      if (rows == 0) continue;
      const int64_t mp = (int64_t)nsmax_ * 2 * nx_;
      if (f == 0)
        (void)rocblas_dgemm_strided_batched(
            h, rocblas_operation_none, rocblas_operation_transpose, 2 * nx_, nsmax_,
            (rocblas_int)rows, &one, b64_.S[0].as<double>(), (rocblas_int)ldS_, rows * ldS_,
            b64_.S[1].as<double>(), (rocblas_int)ldS_, rows * ldS_, &zero,
            static_cast<double*>(work_.get()), 2 * nx_, mp, (rocblas_int)(n_ / rows));
      else
        (void)rocblas_sgemm_strided_batched(
            h, rocblas_operation_none, rocblas_operation_transpose, 2 * nx_, nsmax_,
            (rocblas_int)rows, &onef, b32_.S[0].as<float>(), (rocblas_int)ldS_, rows * ldS_,
            b32_.S[1].as<float>(), (rocblas_int)ldS_, rows * ldS_, &zerof,
            static_cast<float*>(work_.get()), 2 * nx_, mp, (rocblas_int)(n_ / rows));
    }
    LOBPCG_CHECK(rocblas_stop_device_memory_size_query(h, &bytes) == rocblas_status_success,
                 LOBPCG_ERR_HIP, "rocBLAS size query");
    dense_->reserve_library_workspace(bytes);
  }
  // nc_[2]: set by the tridiagonal eigensolver when a QL leaf did not
  // converge; read with n_c once per iteration
  dense_->set_status_word(nc_.as<int32_t>() + 2);
  LOBPCG_HIP(hipHostMalloc((void**)&hbuf_, sizeof(int32_t) * 8, hipHostMallocDefault));
  LOBPCG_HIP(hipHostMalloc((void**)&hdbl_, sizeof(double) * 8, hipHostMallocDefault));
  LOBPCG_HIP(hipEventCreateWithFlags(&ev_nc_, hipEventDisableTiming));
  sketch_norms();
}

// Section 4.3: ||A||_2 >= ||Omega A||_F / ||Omega||_F for a Gaussian Omega
// (n_x x n), here stream 1 of the seeded generator, independent of the initial
// block (a warm start from converged vectors would bias an estimate taken on
// it toward the smallest eigenvalues).  The estimate depends on the operator
// and the seed only, so it is formed once per handle.
void Solver::sketch_norms() {
  const int64_t n = n_;
  const int nx = nx_;
  double* Om = b64_.S[0].as<double>();
  double* AO = b64_.AX.as<double>();
  double* nrm = nrm_.as<double>();
  launch_gaussian(n, nx, Om, ldS_, opt_.seed, kStreamSketch, s_);
  spmm<double>(A_, Om, ldS_, AO, ldX_, nx);
  launch_colsq<double>(n, nx, AO, ldX_, nrm, work_.get(), s_);
  launch_sqrt_sum(nx, nrm, nrm + 4 * nx, s_);
  launch_colsq<double>(n, nx, Om, ldS_, nrm, work_.get(), s_);
  launch_sqrt_sum(nx, nrm, nrm + 4 * nx + 1, s_);
  if (haveB_) {
    spmm<double>(B_, Om, ldS_, AO, ldX_, nx);
    launch_colsq<double>(n, nx, AO, ldX_, nrm, work_.get(), s_);
    launch_sqrt_sum(nx, nrm, nrm + 4 * nx + 2, s_);
  }
  LOBPCG_HIP(hipMemcpyAsync(hdbl_, nrm + 4 * nx, sizeof(double) * 3, hipMemcpyDeviceToHost, s_));
  sync();
  normA_ = hdbl_[0] / hdbl_[1];
  normB_ = haveB_ ? hdbl_[2] / hdbl_[1] : 1.0;
}

Solver::~Solver() {
  if (ev_nc_) (void)hipEventDestroy(ev_nc_);
  if (hbuf_) (void)hipHostFree(hbuf_);
  if (hdbl_) (void)hipHostFree(hdbl_);
}

KernelTimer::~KernelTimer() {
  for (hipEvent_t e : pool_) (void)hipEventDestroy(e);
}

void KernelTimer::enable(bool on) {
  on_ = on;
  if (on) {
    for (auto& t : totals) t = lobpcg_kernel_stat{0, 0.0, 0.0};
    recs_.clear();
    used_ = 0;
  }
}

hipEvent_t KernelTimer::event(size_t i) {
  while (pool_.size() <= i) {
    hipEvent_t e;
    LOBPCG_HIP(hipEventCreate(&e));
    pool_.push_back(e);
  }
  return pool_[i];
}

int KernelTimer::start(hipStream_t s) {
  if (!on_) return -1;
  const int tok = (int)used_++;
  LOBPCG_HIP(hipEventRecord(event(tok), s));
  return tok;
}

void KernelTimer::stop(int token, int kind, double work, hipStream_t s) {
  if (!on_ || token < 0) return;
  const int e1 = (int)used_++;
  LOBPCG_HIP(hipEventRecord(event(e1), s));
  recs_.push_back(Rec{kind, token, e1, work});
  if (used_ > 4096) collect();  // bound the pool
}

void KernelTimer::collect() {
  if (recs_.empty()) {
    used_ = 0;
    return;
  }
  // records can sit on two streams: wait for each of them
  for (const Rec& r : recs_) LOBPCG_HIP(hipEventSynchronize(pool_[r.e1]));
  for (const Rec& r : recs_) {
    float ms = 0.f;
    LOBPCG_HIP(hipEventElapsedTime(&ms, pool_[r.e0], pool_[r.e1]));
    totals[r.kind].launches += 1;
    totals[r.kind].seconds += 1e-3 * ms;
    totals[r.kind].work += r.work;
  }
  recs_.clear();
  used_ = 0;
}

void Solver::sync() { LOBPCG_HIP(hipStreamSynchronize(s_)); }

void Solver::phase_mark(int phase) {
  if (!profile_ || !phase_acc_) {
    cur_phase_ = phase;
    return;
  }
  sync();
  const double t = now_s();
  phase_acc_[cur_phase_] += t - tmark_;
  tmark_ = t;
  cur_phase_ = phase;
}

template <typename T>
void Solver::spmm(const DevCsr& M, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols) {
  if (ncols == 0) return;
  const T* v;
  if constexpr (sizeof(T) == 8) v = M.v64.as<T>();
  else v = M.v32.as<T>();
  const int tok = timer_.start(s_);
  launch_spmm<T>(M.n, M.rowptr.as<int64_t>(), M.colind.as<int32_t>(), v, X, ldx, Y, ldy, ncols, s_);
  const double sv = sizeof(T);
  timer_.stop(tok, 0, (double)M.nnz * (sv + 4) + 8.0 * (M.n + 1) + 2.0 * M.n * ncols * sv, s_);
}

void Solver::apply(bool use_B, const double* X, int64_t ldx, double* Y, int64_t ldy,
                   int ncols) {
  AllocatorScope scope(&alloc_);
  if (use_B && !haveB_) {
    LOBPCG_HIP(hipMemcpy2DAsync(Y, sizeof(double) * ldy, X, sizeof(double) * ldx,
                                sizeof(double) * ncols, n_, hipMemcpyDeviceToDevice, s_));
    return;
  }
  spmm<double>(use_B ? B_ : A_, X, ldx, Y, ldy, ncols);
}

template <typename T>
void Solver::gram(int64_t n, int m, int p, int p1, const T* L, int64_t ldl, const T* R1,
                  int64_t ldr1, const T* R2, int64_t ldr2, double* G1, int c1, double* G2, int c2,
                  int64_t ldg, int mirror_rows) {
  if (m == 0 || p == 0) return;
  const int tok = timer_.start(s_);
  const int64_t rows = gram_library_rows(sizeof(T) == 4, n, m, p);
  if (rows > 0) {
    // Split-K through the library: partial tiles (p x m column-major, i.e.
    // row-major m x p) of equal row chunks by one strided-batched GEMM per R
    // segment (G^T = R^T L in column-major terms), the remainder chunk by a
    // plain GEMM, then the same fixed-order FP64 sum as gram_partial_kernel's.
    rocblas_handle h = dense_->handle();
    T* part = static_cast<T*>(work_.get());
    const int64_t full = n / rows, rem = n - full * rows;
    const int64_t mp = (int64_t)m * p;
    const T one = 1, zero = 0;
    auto gemm = [&](int pr, const T* R, int64_t ldr, int64_t r0, int64_t nr, int64_t batch,
                    T* out) {
      rocblas_status st;
      if constexpr (sizeof(T) == 8)
        st = rocblas_dgemm_strided_batched(
            h, rocblas_operation_none, rocblas_operation_transpose, pr, m, (rocblas_int)nr, &one,
            R + r0 * ldr, (rocblas_int)ldr, nr * ldr, L + r0 * ldl, (rocblas_int)ldl, nr * ldl,
            &zero, out, p, mp, (rocblas_int)batch);
      else
        st = rocblas_sgemm_strided_batched(
            h, rocblas_operation_none, rocblas_operation_transpose, pr, m, (rocblas_int)nr, &one,
            R + r0 * ldr, (rocblas_int)ldr, nr * ldr, L + r0 * ldl, (rocblas_int)ldl, nr * ldl,
            &zero, out, p, mp, (rocblas_int)batch);
      LOBPCG_CHECK(st == rocblas_status_success, LOBPCG_ERR_HIP,
                   "rocBLAS strided-batched GEMM (Gram blocks)");
    };
    const int p2 = p - p1;
    if (full > 0) {
      gemm(p1, R1, ldr1, 0, rows, full, part);
      if (p2 > 0) gemm(p2, R2, ldr2, 0, rows, full, part + p1);
    }
    if (rem > 0) {
      gemm(p1, R1, ldr1, full * rows, rem, 1, part + full * mp);
      if (p2 > 0) gemm(p2, R2, ldr2, full * rows, rem, 1, part + full * mp + p1);
    }
    launch_gram_reduce<T>(m, p, p1, (int)(full + (rem > 0)), part, G1, c1, G2, c2, ldg,
                          mirror_rows, s_);
  } else {
    launch_gram<T>(n, m, p, p1, L, ldl, R1, ldr1, R2, ldr2, G1, c1, G2, c2, ldg, mirror_rows,
                   work_.get(), s_);
  }
  timer_.stop(tok, 1, 2.0 * n * m * p, s_);
}

// The basis update Y = S C is a plain GEMM.  Measured on MI355X: rocBLAS's
// GEMM runs the FP32 products at 67-144 TFLOP/s against 54-71 for
// update_kernel (64^3 to 96^3 shapes, K = 330-3300, N = 110-1100), and the
// FP64 ones at 61-72 against 55-59 once K * N reaches ~5e5, while
// update_kernel is the faster one for the FP64 shapes of the 64^3 workload
// (K = 330, N <= 220: 50-52 against 40-49).
static bool update_uses_library(bool fp32, int K, int N) {
  if (fp32) return true;
  return (int64_t)K * N >= 250000;
}

template <typename T>
void Solver::update(int64_t n, int K, int N, const T* S, int64_t lds, const double* C,
                    int64_t ldc, double alpha, double beta, T* Y, int64_t ldy,
                    hipStream_t stream) {
  if (N == 0) return;
  // another stream takes the hand-written kernel only (the library route's
  // handle and FP32 copy of C belong to the main stream)
  LOBPCG_CHECK(!stream || !update_uses_library(sizeof(T) == 4, K, N), LOBPCG_ERR_ARG,
               "update: the library route runs on the main stream");
  const hipStream_t us = stream ? stream : s_;
  const int tok = timer_.start(us);
  if (update_uses_library(sizeof(T) == 4, K, N)) {
    // Y^T (N x n) = C^T (N x K) S^T (K x n) in column-major terms: S, Y row-major
    rocblas_handle h = dense_->handle();
    if constexpr (sizeof(T) == 4) {
      launch_copy2d<double, float>(N, K, C, ldc, C32_.as<float>(), ldc, s_);
      const float a = (float)alpha, b = (float)beta;
      LOBPCG_CHECK(rocblas_sgemm(h, rocblas_operation_transpose, rocblas_operation_none, N,
                                 (rocblas_int)n, K, &a, C32_.as<float>(), (rocblas_int)ldc, S,
                                 (rocblas_int)lds, &b, Y, (rocblas_int)ldy) ==
                       rocblas_status_success,
                   LOBPCG_ERR_HIP, "rocblas_sgemm (basis update)");
    } else {
      LOBPCG_CHECK(rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, N,
                                 (rocblas_int)n, K, &alpha, C, (rocblas_int)ldc, S,
                                 (rocblas_int)lds, &beta, Y, (rocblas_int)ldy) ==
                       rocblas_status_success,
                   LOBPCG_ERR_HIP, "rocblas_dgemm (basis update)");
    }
  } else {
    launch_update<T>(n, K, N, S, lds, C, ldc, alpha, beta, Y, ldy, us);
  }
  timer_.stop(tok, 2, 2.0 * n * K * N, us);
}

// Algorithm 5 (orthoDrop) with Algorithms 4 (svqb) and 6 (svqbDrop), metric
// M = B (or I).  U: n x nu (ldu) in place; V: n x nv (ldv) M-orthonormal external
// basis with MV = M V (ldmv).  M U is recomputed explicitly after every inner
// pass (section 5.2: no implicit products inside orthogonalisation).  Returns the
// number of columns kept.
template <typename T>
int Solver::ortho_drop(Blocks<T>& b, const DevCsr* B, T* U, int64_t ldu, int nu, const T* V,
                       int64_t ldv, const T* MV, int64_t ldmv, int nv, double tau_ortho,
                       double eps, lobpcg_info* info) {
  if (info) info->ortho_calls++;
  const int64_t ldg = nsmax_;
  double* G = GB_.as<double>();        // scratch: Gram of U (nu x nu)
  double* Gv = GA_.as<double>();       // scratch: V^T M U (nv x nu)
  double* Tu = C_.as<double>();        // svqb transform (nu x nkeep, ld nu)
  double* nrm = nrm_.as<double>();
  // device slots read back together once per inner pass:
  //   t[0] ||U^T M U - I||_F, t[1] ||U||_F, t[2] ||MU||_F, t[3] ||V^T M U||_F, t[4] ||MV||_F
  double* t = nrm + 4 * nx_;
  T* U2 = b.U2.template as<T>();
  T* MU = B ? b.MU.template as<T>() : U;
  const int64_t ldmu = B ? ldX_ : ldu;
  if (nv > 0) {
    launch_colsq<T>(n_, nv, MV, ldmv, nrm, work_.get(), s_);
    launch_sqrt_sum(nv, nrm, t + 4, s_);
  }
  auto gram_u = [&]() {
    if (B) spmm<T>(*B, U, ldu, MU, ldmu, nu);
    gram<T>(n_, nu, nu, nu, U, ldu, MU, ldmu, nullptr, 0, G, 0, nullptr, 0, ldg, 0);
  };
  double outer_err = 0.0;
  for (int i = 0; i < 3 && nu > 0; ++i) {
    // Outer pass: U = U - V (V^T M U) (block classical Gram-Schmidt).
    if (nv > 0) {
      gram<T>(n_, nv, nu, nu, MV, ldmv, U, ldu, nullptr, 0, Gv, 0, nullptr, 0, ldg, 0);
      update<T>(n_, nv, nu, V, ldv, Gv, ldg, -1.0, 1.0, U, ldu);
    }
    gram_u();
    for (int j = 0; j < 3 && nu > 0; ++j) {
      // Inner passes: svqb on the first, svqbDrop afterwards (Algorithm 3,
      // ortho_mode 1: svqb on every pass, nothing dropped).
      const bool drop = j > 0 && opt_.ortho_mode == 0;
      const double factor = drop ? (opt_.drop_factor > 0 ? opt_.drop_factor : 10.0)
                                 : (opt_.replace_factor > 0 ? opt_.replace_factor : 10.0);
      const double tau = factor * nu * eps;
      const int keep = dense_->svqb_transform(G, ldg, nu, tau, drop, Tu);
      if (info) info->svqb_calls++;
      if (keep == 0) return 0;
      update<T>(n_, nu, keep, U, ldu, Tu, nu, 1.0, 0.0, U2, ldX_);
      launch_copy2d<T, T>(n_, keep, U2, ldX_, U, ldu, s_);
      nu = keep;
      // Inner test ||U^T M U - I|| / (||MU|| ||U||) with MU recomputed, and the
      // outer test ||V^T M U|| / (||MV|| ||U||) on the same U, read back together
      // (the outer value is used only when this inner pass ends the inner loop).
      gram_u();
      launch_fro_minus_identity(nu, G, ldg, t, s_);
      launch_colsq<T>(n_, nu, U, ldu, nrm, work_.get(), s_);
      launch_sqrt_sum(nu, nrm, t + 1, s_);
      launch_colsq<T>(n_, nu, MU, ldmu, nrm, work_.get(), s_);
      launch_sqrt_sum(nu, nrm, t + 2, s_);
      if (nv > 0) {
        gram<T>(n_, nv, nu, nu, MV, ldmv, U, ldu, nullptr, 0, Gv, 0, nullptr, 0, ldg, 0);
        launch_fro(nv, nu, Gv, ldg, t + 3, s_);
      }
      LOBPCG_HIP(hipMemcpyAsync(hdbl_, t, sizeof(double) * 5, hipMemcpyDeviceToHost, s_));
      sync();
      outer_err = nv > 0 ? hdbl_[3] / (hdbl_[4] * hdbl_[1]) : 0.0;
      const double err = hdbl_[0] / (hdbl_[2] * hdbl_[1]);
      if (err <= tau_ortho) break;
    }
    if (nv == 0 || nu == 0) break;
    if (outer_err <= tau_ortho) break;
  }
  return nu;
}

template <typename T>
int Solver::run(Blocks<T>& b, const DevCsr& A, const DevCsr* B, double tol, int maxit,
                const double* X0dev, double tau_skip, double tau_ortho, lobpcg_precond_fn K,
                void* Kuser, lobpcg_info* info, int* iters_out) {
  const int64_t n = n_;
  const int nx = nx_;
  const int64_t ldS = ldS_, ldX = ldX_, ldBXP = 2 * ldX_;
  const int64_t ldg = nsmax_, ldc = nsmax_;
  const double eps = sizeof(T) == 8 ? kEps64 : kEps32;
  const bool lq_literal = opt_.lq_literal != 0;
  const bool use_cb = opt_.precond == 2 && K != nullptr;
  const double* dinv = opt_.precond == 1 ? dinv_.as<double>() : nullptr;
  double* GA = GA_.as<double>();
  double* GB = GB_.as<double>();
  double* C = C_.as<double>();
  double* theta = theta_.as<double>();
  double* theta_p = theta_p_.as<double>();
  // With implicit product updates (section 5.2, B = I) A X, A P and A W live in
  // AS[cur] with the column layout of S and A X, A P follow the basis update
  // (A S C); otherwise A X is recomputed with the sparse product.
  const bool impl = opt_.implicit_products == 1;
  auto ASp = [&](int which) -> T* { return b.AS[which].template as<T>(); };
  T* AX = b.AX.template as<T>();
  int64_t ldAX = ldX;
  T* AW = b.AW.template as<T>();
  T* BXP = B ? b.BXP.template as<T>() : nullptr;
  T* BW = B ? b.BW.template as<T>() : nullptr;
  T* Rb = b.R.template as<T>();
  int cur = 0;
  *iters_out = 0;
  int np = 0, nc = 0;
  int rc = LOBPCG_NOT_CONVERGED;
  int it = 0;
  bool have_x = false;  // S[cur] holds a Rayleigh-Ritz block X
  int nc_best = 0, it_best = 0;  // FP32 phase: last iteration that raised n_c
  try {
  // Algorithm 8's start: Rayleigh-Ritz on X0 (Algorithm 2), X = X0 C.
  phase_mark(7);
  LOBPCG_HIP(hipMemsetAsync(nc_.get(), 0, sizeof(int32_t) * 4, s_));
  T* S0 = b.S[0].template as<T>();
  launch_copy2d<double, T>(n, nx, X0dev, nx, S0, ldS, s_);
  phase_mark(0);
  spmm<T>(A, S0, ldS, AX, ldX, nx);
  if (B) spmm<T>(*B, S0, ldS, BXP, ldBXP, nx);
  phase_mark(3);
  gram<T>(n, nx, 2 * nx, nx, S0, ldS, AX, ldX, B ? BXP : S0, B ? ldBXP : ldS, GA, 0, GB, 0,
                 ldg, 0);
  phase_mark(4);
  RROutput o0 = dense_->rr_modified(GA, GB, ldg, nx, nx, 0, false, false, 0.0, C, ldc, theta,
                                    theta_p, nx);
  if (o0.flipped)
    throw Error(LOBPCG_ERR_BREAKDOWN,
                "Cholesky of the initial block's Gram matrix failed (potrf info " +
                    std::to_string(o0.potrf_info) + ", trtri info " + std::to_string(o0.trtri_info) +
                    ", cond " + std::to_string(o0.cond) + ")");
  phase_mark(5);
  T* S1 = b.S[1].template as<T>();
  update<T>(n, nx, nx, S0, ldS, C, ldc, 1.0, 0.0, S1, ldS);
  cur = 1;
  have_x = true;
  // First residual R = AX - BX Theta; W = K^-1 R stored reversed after X (P is empty).
  phase_mark(0);
  if (impl) {
    AX = ASp(cur);
    ldAX = ldS;
  }
  spmm<T>(A, S1, ldS, AX, ldAX, nx);
  if (B) spmm<T>(*B, S1, ldS, BXP, ldBXP, nx);
  phase_mark(6);
  launch_residual<T>(n, nx, AX, ldAX, B ? BXP : nullptr, ldBXP, S1, ldS, theta, dinv,
                     use_cb ? Rb : S1 + nx, use_cb ? ldX : ldS, normA_, normB_, tol,
                     rho_.as<double>(), nc_.as<int32_t>(), work_.get(), s_);
  // useOrtho starts false, or true from the start in the versions of
  // section 6 that orthogonalise every iteration
  // Algorithm 1 (basic): no orthogonalisation, no locking of W, explicit Gram
  // blocks, Algorithm 2's Rayleigh-Ritz, and its own P
  const bool basic = opt_.basic != 0;
  bool use_ortho = !basic && opt_.force_ortho != 0;
  // The implicit X and P blocks (eqs. (12)-(14)) take [X P] as exactly
  // B-orthonormal.  A Cholesky-based step leaves it so only to about
  // eps cond(R)^2, and these errors compound from step to step while the
  // cond(R) test, which sees the assumed identity block, stays blind to them:
  // a long run with tiny residuals (cond(R) of 1e3-1e5 for tens of steps)
  // can drift to O(1e-2) and lose eigenvectors.  After a step whose cond(R)
  // exceeded tau_skip^(-1/4) (FP64: 4.6e3, at most about sqrt(eps / 10) of
  // orthonormality error per step), the next step forms the X and P blocks
  // explicitly, so that its factor and condition test see S^T B S itself.
  const double cond_xp = tau_skip > 0.0 ? std::pow(tau_skip, -0.25) : HUGE_VAL;
  bool xp_explicit = false;
  for (it = 1; it <= maxit; ++it) {
    T* Sc = b.S[cur].template as<T>();
    T* Sn = b.S[cur ^ 1].template as<T>();
    const int nv = nx + np;
    T* W = Sc + nv;
    int nw = basic ? nx : nx - nc;
    T* AWc = impl ? ASp(cur) + nv : AW;
    const int64_t ldAW = impl ? ldS : ldX;
    // W from the residual with the preconditioner applied (W0 = K^-1 R).
    if (use_cb) {
      phase_mark(1);
      const int st = K(Kuser, n, nw, sizeof(T) == 8 ? 0 : 1, Rb, ldX, W, ldS, (void*)s_);
      if (st != 0) throw Error(LOBPCG_ERR_CALLBACK, "preconditioner callback returned nonzero");
    }
    const T* MV = B ? BXP : Sc;
    const int64_t ldmv = B ? ldBXP : ldS;
    if (use_ortho) {
      phase_mark(5);
      dense_->join_p();  // P, updated on the second stream, is read from here on
      phase_mark(2);
      nw = ortho_drop<T>(b, B, W, ldS, nw, Sc, ldS, MV, ldmv, nv, tau_ortho, eps, info);
    }
    RROutput o;
    for (int attempt = 0; attempt < 2; ++attempt) {
      const int ns = nv + nw;
      // A W and B W (explicit: every block involving W is computed, section 5.2).
      phase_mark(0);
      spmm<T>(A, W, ldS, AWc, ldAW, nw);
      if (B) spmm<T>(*B, W, ldS, BW, ldX, nw);
      phase_mark(5);
      dense_->join_p();  // the Gram reads P, updated on the second stream
      // Gram columns of W in S^T A S and S^T B S; the rest from eqs. (12)-(14).
      phase_mark(3);
      gram<T>(n, ns, use_ortho ? nw : 2 * nw, nw, Sc, ldS, AWc, ldAW, B ? BW : W,
              B ? ldX : ldS, GA, nv, GB, nv, ldg, nv);
      const bool implicit_xp = opt_.implicit_gram && !basic && !xp_explicit;
      if (info && attempt == 0 && opt_.implicit_gram && !basic && xp_explicit)
        info->explicit_xp_steps++;
      if (implicit_xp) {
        launch_fill_implicit(nx, np, theta, theta_p, nx, GA, use_ortho ? nullptr : GB, ldg, s_);
      } else {
        // The X and P blocks computed explicitly: [X P]^T [AX AP] and
        // [X P]^T [BX BP] (or [X P]^T [X P]); A P from the implicit update, or
        // by the sparse product through the ortho buffer.
        T* AP = impl ? ASp(cur) + nx : b.U2.template as<T>();
        const int64_t ldAP = impl ? ldS : ldX;
        phase_mark(0);
        if (np > 0 && !impl) spmm<T>(A, Sc + nx, ldS, AP, ldAP, np);
        phase_mark(3);
        gram<T>(n, nv, nv, nx, Sc, ldS, AX, ldAX, AP, ldAP, GA, 0, GA, nx, ldg, 0);
        if (!use_ortho)
          gram<T>(n, nv, nv, nv, Sc, ldS, B ? BXP : Sc, B ? ldBXP : ldS, nullptr, 0, GB, 0,
                  nullptr, 0, ldg, 0);
      }
      // RayleighRitzModified (Algorithm 7); its P block is left running on the second
      // stream beside the X update, A X and the residual, which do not touch P.
      phase_mark(4);
      {
        const int tok = timer_.start(s_);
        // with the implicit blocks the X/P block of S^T B S is exactly I
        o = dense_->rr_modified(GA, GB, ldg, ns, nx, nc, use_ortho, lq_literal,
                                basic ? 0.0 : tau_skip, C, ldc, theta, theta_p, nx, !basic,
                                implicit_xp ? nv : 0, basic);
        timer_.stop(tok, 4, 0.0, s_);
      }
      if (!o.flipped) break;
      if (basic)
        throw Error(LOBPCG_ERR_BREAKDOWN,
                    "Algorithm 1: S^T B S has no Cholesky factor (basic LOBPCG broke down)");
      // Cholesky rejected: switch to orthogonalised W for good and redo the step.
      use_ortho = true;
      if (info) {
        info->flips++;
        if (info->ortho_switch_iter < 0) info->ortho_switch_iter = info->iterations + it;
      }
      phase_mark(2);
      nw = ortho_drop<T>(b, B, W, ldS, nw, Sc, ldS, MV, ldmv, nv, tau_ortho, eps, info);
    }
    if (o.flipped) throw Error(LOBPCG_ERR_BREAKDOWN, "Rayleigh-Ritz failed after orthoDrop");
    xp_explicit = !use_ortho && o.cond > cond_xp;
    const int ns = nv + nw;
    const int npn = o.np;
    // Basis update [X, P] = S [C_x, C_p]: X now, P once the P block is done.
    phase_mark(5);
    update<T>(n, ns, nx, Sc, ldS, C, ldc, 1.0, 0.0, Sn, ldS);
    T* ASo = impl ? ASp(cur) : nullptr;
    cur ^= 1;
    // Residual R = AX - BX Theta with A X recomputed by the sparse product, or
    // updated implicitly as A X = (A S) C_x (section 5.2).
    // With B = I and A X recomputed, the sparse product and the residual run
    // as one kernel (A X is stored only when the next step forms its X/P Gram
    // blocks explicitly, the one later use).
    const bool fused = !impl && !B;
    if (impl) {
      AX = ASp(cur);
      update<T>(n, ns, nx, ASo, ldS, C, ldc, 1.0, 0.0, AX, ldS);
    } else if (!fused) {
      phase_mark(0);
      spmm<T>(A, Sn, ldS, AX, ldX, nx);
    }
    if (B) spmm<T>(*B, Sn, ldS, BXP, ldBXP, nx);
    phase_mark(6);
    if (fused) {
      const bool keep_ax = !opt_.implicit_gram || basic || xp_explicit;
      const T* av;
      if constexpr (sizeof(T) == 8) av = A.v64.as<T>();
      else av = A.v32.as<T>();
      const double sv = sizeof(T);
      const int tok = timer_.start(s_);
      launch_spmm_residual<T>(n, A.rowptr.as<int64_t>(), A.colind.as<int32_t>(), av, Sn, ldS,
                              nx, theta, dinv, use_cb ? Rb : Sn + nx + npn,
                              use_cb ? ldX : ldS, keep_ax ? AX : nullptr, ldAX, normA_, tol,
                              rho_.as<double>(), nc_.as<int32_t>(), work_.get(), s_);
      timer_.stop(tok, 0,
                  (double)A.nnz * (sv + 4) + 8.0 * (n + 1) + (double)n * nx * sv * (keep_ax ? 3 : 2) +
                      (dinv ? 8.0 * n : 0.0),
                  s_);
    } else {
      const int tok = timer_.start(s_);
      launch_residual<T>(n, nx, AX, ldAX, B ? BXP : nullptr, ldBXP, Sn, ldS, theta, dinv,
                         use_cb ? Rb : Sn + nx + npn, use_cb ? ldX : ldS, normA_, normB_, tol,
                         rho_.as<double>(), nc_.as<int32_t>(), work_.get(), s_);
      timer_.stop(tok, 3, (double)n * nx * sizeof(T) * (B ? 4 : 3) + (dinv ? 8.0 * n : 0.0), s_);
    }
    // Number of converged pairs (leading run meeting criterion 9); the
    // host waits for this copy only, the P update runs on meanwhile.
    LOBPCG_HIP(hipMemcpyAsync(hbuf_, nc_.get(), sizeof(int32_t) * 3, hipMemcpyDeviceToHost, s_));
    LOBPCG_HIP(hipEventRecord(ev_nc_, s_));
    // P = S C_p.  FP64 with the hand-written kernel, B = I and A P not updated:
    // queued behind Algorithm 7's P block on the second stream, so that it runs
    // beside the next step's A W; that step joins before its first read of P
    // (orthoDrop or the Gram).  Otherwise the main stream waits for the P block
    // (Rayleigh-Ritz time) and updates.
    const hipStream_t ps = dense_->p_stream();
    if (npn > 0 && ps && sizeof(T) == 8 && !impl && !B &&
        !update_uses_library(false, ns, npn)) {
      update<T>(n, ns, npn, Sc, ldS, C + (int64_t)nx * ldc, ldc, 1.0, 0.0, Sn + nx, ldS, ps);
      dense_->extend_p();
    } else {
      phase_mark(4);
      dense_->join_p();
      phase_mark(5);
      if (npn > 0) {
        update<T>(n, ns, npn, Sc, ldS, C + (int64_t)nx * ldc, ldc, 1.0, 0.0, Sn + nx, ldS);
        if (impl)
          update<T>(n, ns, npn, ASo, ldS, C + (int64_t)nx * ldc, ldc, 1.0, 0.0, AX + nx, ldS);
        if (B) spmm<T>(*B, Sn + nx, ldS, BXP + nx, ldBXP, npn);
      }
    }
    np = npn;
    LOBPCG_HIP(hipEventSynchronize(ev_nc_));
    if (hbuf_[2] == 2)
      throw Error(LOBPCG_ERR_NONFINITE, "non-finite projected matrix");
    if (hbuf_[2])
      throw Error(LOBPCG_ERR_BREAKDOWN,
                  "projected eigenproblem: an implicit QL leaf of the tridiagonal "
                  "divide and conquer did not converge");
    if (hbuf_[1]) throw Error(LOBPCG_ERR_NONFINITE, "non-finite Ritz value or residual");
    nc = hbuf_[0];
    if (opt_.progress)
      opt_.progress(opt_.progress_user, (info ? info->iterations : 0) + it, nc,
                    sizeof(T) == 4 ? 1 : 0);
    if (nc >= k_) {
      rc = LOBPCG_OK;
      break;
    }
    if constexpr (sizeof(T) == 4) {
      // The FP32 phase hands over once it stops making progress: when no
      // further pair has met the FP32 threshold for kFp32StallIters iterations
      // (its Gram blocks carry FP32 rounding, which sets a residual floor).
      if (fp32_soft_) {
        if (nc > nc_best) {
          nc_best = nc;
          it_best = it;
        } else if (it - it_best >= kFp32StallIters) {
          fp32_stalled_ = true;
          break;
        }
      }
    }
    if (nx - nc == 0 && np == 0) throw Error(LOBPCG_ERR_BREAKDOWN, "search space collapsed");
  }
  dense_->join_p();  // a P update still queued on the second stream
  } catch (const Error& e) {
    // A breakdown or a non-finite value in the FP32 phase of the precision
    // split does not end the solve: the FP64 phase takes over, from the last
    // block X when it is finite (breakdown) or from the initial block
    // (non-finite values), which X0buf still holds.
    const bool recoverable = e.code == LOBPCG_ERR_BREAKDOWN || e.code == LOBPCG_ERR_NONFINITE;
    if (sizeof(T) != 4 || !recoverable || !fp32_soft_) throw;
    dense_->join_p();
    phase_mark(7);
    fp32_failure_ = e.what();
    *iters_out = std::min(it, maxit);
    final_nc_ = 0;
    if (e.code == LOBPCG_ERR_BREAKDOWN && have_x) {
      const T* Xc = b.S[cur].template as<T>();
      double* nrm = nrm_.as<double>();
      launch_colsq<T>(n, nx, Xc, ldS, nrm, work_.get(), s_);
      launch_sqrt_sum(nx, nrm, nrm + 4 * nx, s_);
      LOBPCG_HIP(hipMemcpyAsync(hdbl_, nrm + 4 * nx, sizeof(double), hipMemcpyDeviceToHost, s_));
      sync();
      if (std::isfinite(hdbl_[0]))
        launch_copy2d<T, double>(n, nx, Xc, ldS, X0buf_.as<double>(), nx, s_);
    }
    return e.code;
  }
  phase_mark(7);
  *iters_out = std::min(it, maxit);
  final_nc_ = nc;
  // Remember where X lives.
  if constexpr (sizeof(T) == 8) {
    Xres_ = b.S[cur].template as<double>();
  } else {
    launch_copy2d<float, double>(n, nx, b.S[cur].template as<float>(), ldS, X0buf_.as<double>(),
                                 nx, s_);
  }
  return rc;
}

int Solver::solve(double tol, const double* X0, bool x0_dev, lobpcg_precond_fn K, void* Kuser,
                  lobpcg_info* info) {
  LOBPCG_CHECK(tol > 0.0, LOBPCG_ERR_ARG, "tol must be positive");
  LOBPCG_CHECK(opt_.precond != 2 || K != nullptr, LOBPCG_ERR_ARG,
               "precond = 2 needs a callback");
  AllocatorScope scope(&alloc_);
  lobpcg_info local{};
  lobpcg_info* inf = info ? info : &local;
  std::memset(inf, 0, sizeof(*inf));
  inf->ortho_switch_iter = -1;
  phase_acc_ = inf->seconds_phase;
  tmark_ = now_s();
  cur_phase_ = 7;
  const double t0 = now_s();
  solved_ = false;
  const int64_t n = n_;
  const int nx = nx_;
  double* X0b = X0buf_.as<double>();
  if (X0 == nullptr) {
    launch_gaussian(n, nx, X0b, nx, opt_.seed, kStreamInitialBlock, s_);
  } else {
    LOBPCG_HIP(hipMemcpyAsync(X0b, X0, sizeof(double) * n * nx,
                              x0_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s_));
  }
  inf->norm_A_est = normA_;
  inf->norm_B_est = normB_;
  const int maxit = opt_.maxit > 0 ? opt_.maxit : 2000;
  const double skip = opt_.skip_factor > 0 ? opt_.skip_factor : 10.0;
  const DevCsr* B = haveB_ ? &B_ : nullptr;
  int rc = LOBPCG_OK;
  int iters = 0;
  if (opt_.precision == 1) {
    const double tol32 = std::max(opt_.fp32_tol > 0 ? opt_.fp32_tol : 1e-5, tol);
    fp32_soft_ = true;
    fp32_stalled_ = false;
    try {
      rc = run<float>(b32_, A_, B, tol32, maxit, X0b, skip * kEps32, 1e-5, K, Kuser, inf, &iters);
    } catch (...) {
      fp32_soft_ = false;
      throw;
    }
    fp32_soft_ = false;
    inf->fp32_iterations = iters;
    inf->iterations = iters;
    if (rc < 0) inf->fp32_fallback = 1;
    if (fp32_stalled_) inf->fp32_fallback = 2;
    // FP64 refinement: Algorithm 8 again, started from the FP32 block (now in X0buf).
    const int left = std::max(1, maxit - iters);
    rc = run<double>(b64_, A_, B, tol, left, X0b, skip * kEps64,
                     opt_.tau_ortho > 0 ? opt_.tau_ortho : 1e-12, K, Kuser, inf, &iters);
    inf->fp64_iterations = iters;
    inf->iterations += iters;
  } else {
    rc = run<double>(b64_, A_, B, tol, maxit, X0b, skip * kEps64,
                     opt_.tau_ortho > 0 ? opt_.tau_ortho : 1e-12, K, Kuser, inf, &iters);
    inf->fp64_iterations = iters;
    inf->iterations = iters;
  }
  sync();
  timer_.collect();
  inf->n_converged = final_nc_;
  inf->seconds_total = now_s() - t0;
  phase_acc_ = nullptr;
  solved_ = true;
  return rc;
}

int Solver::eigpairs(int count, double* lambda, double* X, int64_t ldx, double* rho,
                     bool on_device) {
  LOBPCG_CHECK(solved_, LOBPCG_ERR_STATE, "eigpairs called before a successful solve");
  LOBPCG_CHECK(count >= 0 && count <= nx_, LOBPCG_ERR_ARG, "count must be in [0, n_x]");
  if (count == 0) return LOBPCG_OK;
  const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  const bool neg = opt_.largest != 0;
  if (lambda && neg && on_device) {
    launch_negate(count, theta_.as<double>(), lambda, s_);
  } else if (lambda) {
    LOBPCG_HIP(hipMemcpyAsync(lambda, theta_.get(), sizeof(double) * count, kind, s_));
  }
  if (rho) LOBPCG_HIP(hipMemcpyAsync(rho, rho_.get(), sizeof(double) * count, kind, s_));
  if (X) {
    LOBPCG_CHECK(ldx >= count, LOBPCG_ERR_ARG, "ldx < count");
    LOBPCG_HIP(hipMemcpy2DAsync(X, sizeof(double) * ldx, Xres_, sizeof(double) * ldS_,
                                sizeof(double) * count, n_, kind, s_));
  }
  sync();
  if (lambda && neg && !on_device)
    for (int i = 0; i < count; ++i) lambda[i] = -lambda[i];
  return LOBPCG_OK;
}

template int Solver::run<double>(Blocks<double>&, const DevCsr&, const DevCsr*, double, int,
                                 const double*, double, double, lobpcg_precond_fn, void*,
                                 lobpcg_info*, int*);
template int Solver::run<float>(Blocks<float>&, const DevCsr&, const DevCsr*, double, int,
                                const double*, double, double, lobpcg_precond_fn, void*,
                                lobpcg_info*, int*);
template struct Blocks<double>;
template struct Blocks<float>;

}  // namespace lobpcg
