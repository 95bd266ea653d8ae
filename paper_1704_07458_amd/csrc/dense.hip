// FP64 projected-problem routines on the device (Algorithms 2, 4, 6, 7).
#include "dense.hpp"

#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "kernels.hpp"
#include "cholinv.hpp"
#include "small_gemm.hpp"
#include "tridiag_dc.hpp"

namespace lobpcg {

#define LOBPCG_ROCBLAS(call)                                                               \
  do {                                                                                     \
    rocblas_status st_ = (call);                                                           \
    if (st_ != rocblas_status_success)                                                     \
      throw ::lobpcg::Error(LOBPCG_ERR_HIP, std::string(#call) + ": " +                    \
                                                rocblas_status_to_string(st_));            \
  } while (0)

// The internal leading dimension is even: the tridiagonalisation then reads
// rows in 16-byte pairs.
Dense::Dense(int nsmax, int nxmax, hipStream_t s)
    : nsmax_(nsmax + (nsmax & 1)), nxmax_(nxmax), s_(s) {
  kTridiagMaxN = std::min(sytrd_max_n(), tridiag_dc_max_n());
  LOBPCG_ROCBLAS(rocblas_create_handle(&h_));
  LOBPCG_ROCBLAS(rocblas_set_stream(h_, s_));
  // Reproducible results: no split-K GEMM kernels that accumulate with
  // atomics (run-to-run rounding differences would change the iteration).
  LOBPCG_ROCBLAS(rocblas_set_atomics_mode(h_, rocblas_atomics_not_allowed));
  // The second stream keeps the default priority; it never blocks on the
  // main stream implicitly (events order the two).
  LOBPCG_HIP(hipStreamCreateWithFlags(&s2_, hipStreamNonBlocking));
  LOBPCG_ROCBLAS(rocblas_create_handle(&h2_));
  LOBPCG_ROCBLAS(rocblas_set_stream(h2_, s2_));
  LOBPCG_ROCBLAS(rocblas_set_atomics_mode(h2_, rocblas_atomics_not_allowed));
  for (hipEvent_t* e : {&ev_z_, &ev_p_})
    LOBPCG_HIP(hipEventCreateWithFlags(e, hipEventDisableTiming));
  const size_t sq = sizeof(double) * (size_t)nsmax_ * nsmax_;
  H_.alloc(sq);
  R_.alloc(sq);
  Ri_.alloc(sq);
  T1_.alloc(sq);
  Mt_.alloc(sq);
  ZQ_.alloc(sq);
  Qs_.alloc(sq);
  d_.alloc(sizeof(double) * nsmax_);
  E_.alloc(sizeof(double) * 2 * nsmax_);
  tau_.alloc(sizeof(double) * nsmax_);
  th2_.alloc(sizeof(double) * nsmax_);
  scale_.alloc(sizeof(double) * nsmax_);
  info_.alloc(sizeof(int32_t) * 8);
  LOBPCG_HIP(hipMemsetAsync(info_.get(), 0, sizeof(int32_t) * 8, s_));
  cond_.alloc(sizeof(double) * 2);
  sinfo_.alloc(sizeof(int32_t) * 2);
  dcY_.alloc(sq);
  dcv_.alloc(sizeof(double) * 4 * nsmax_);
  dci_.alloc(sizeof(int32_t) * tridiag_dc_int_workspace());
  dcw_.alloc(sizeof(double) * 2 * tridiag_dc_max_n());
  dcr_.alloc(sizeof(double) * 64);
  LOBPCG_HIP(hipHostMalloc((void**)&hinfo_, sizeof(int32_t) * 8, hipHostMallocDefault));
  LOBPCG_HIP(hipHostMalloc((void**)&hcond_, sizeof(double) * 2, hipHostMallocDefault));
  // The library routines' device workspace comes from this object's allocator
  // too: size it for the largest projected problem, then hand it to the handles.
  lib_ws_.alloc(library_workspace_bytes(h_));
  LOBPCG_ROCBLAS(rocblas_set_workspace(h_, lib_ws_.get(), lib_ws_.size()));
  lib_ws2_.alloc(library_workspace_bytes(h2_));
  LOBPCG_ROCBLAS(rocblas_set_workspace(h2_, lib_ws2_.get(), lib_ws2_.size()));
}

// Device workspace the rocBLAS / rocSOLVER calls of this object need at the
// largest sizes (their device-memory size query); the buffers passed are real
// ones of the right sizes, nothing is computed.
size_t Dense::library_workspace_bytes(rocblas_handle h) {
  const int n = nsmax_;
  const int64_t ld = nsmax_;
  double* A = H_.as<double>();
  double* w = d_.as<double>();
  double* e = E_.as<double>();
  int32_t* info = info_.as<int32_t>();
  size_t bytes = 0;
  LOBPCG_ROCBLAS(rocblas_start_device_memory_size_query(h));
  (void)rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, n, A, (rocblas_int)ld, w,
                         e, info);
  (void)rocsolver_dstedc(h, rocblas_evect_tridiagonal, n, w, e, A, (rocblas_int)ld, info);
  (void)rocsolver_dpotrf(h, rocblas_fill_upper, n, A, (rocblas_int)ld, info);
  (void)rocsolver_dtrtri(h, rocblas_fill_upper, rocblas_diagonal_non_unit, n, A, (rocblas_int)ld,
                         info);
  (void)rocsolver_dgeqrf(h, n, nxmax_, A, (rocblas_int)ld, tau_.as<double>());
  (void)rocsolver_dorgqr(h, n, nxmax_, nxmax_, A, (rocblas_int)ld, tau_.as<double>());
  const double one = 1.0, zero = 0.0;
  (void)rocblas_dgemm(h, rocblas_operation_transpose, rocblas_operation_none, n, n, n, &one, A,
                      (rocblas_int)ld, A, (rocblas_int)ld, &zero, R_.as<double>(), (rocblas_int)ld);
  (void)rocblas_dgeam(h, rocblas_operation_transpose, rocblas_operation_none, n, n, &one, A,
                      (rocblas_int)ld, &zero, R_.as<double>(), (rocblas_int)ld, R_.as<double>(),
                      (rocblas_int)ld);
  LOBPCG_ROCBLAS(rocblas_stop_device_memory_size_query(h, &bytes));
  return std::max<size_t>(bytes, 256);
}

void Dense::reserve_library_workspace(size_t bytes) {
  if (bytes <= lib_ws_.size()) return;
  LOBPCG_HIP(hipStreamSynchronize(s_));
  lib_ws_.alloc(bytes);
  LOBPCG_ROCBLAS(rocblas_set_workspace(h_, lib_ws_.get(), lib_ws_.size()));
}

Dense::~Dense() {
  if (s2_) (void)hipStreamSynchronize(s2_);
  for (hipEvent_t e : {ev_z_, ev_p_})
    if (e) (void)hipEventDestroy(e);
  if (h2_) rocblas_destroy_handle(h2_);
  if (s2_) (void)hipStreamDestroy(s2_);
  if (h_) rocblas_destroy_handle(h_);
  if (hinfo_) (void)hipHostFree(hinfo_);
  if (hcond_) (void)hipHostFree(hcond_);
}

// Products of the projected-problem sizes go to the MFMA small-product kernel on
// the handle's stream (a library GEMM uses a handful of workgroups there);
// larger ones to rocBLAS.
static void dgemm(rocblas_handle h, rocblas_operation ta, rocblas_operation tb, int m, int n,
                  int k, double alpha, const double* A, int64_t lda, const double* B, int64_t ldb,
                  double beta, double* C, int64_t ldc) {
  if (m == 0 || n == 0) return;
  if (small_dgemm_fits(m, n, k)) {
    hipStream_t s = nullptr;
    LOBPCG_ROCBLAS(rocblas_get_stream(h, &s));
    small_dgemm(ta == rocblas_operation_transpose, tb == rocblas_operation_transpose, m, n, k,
                alpha, A, lda, B, ldb, beta, C, ldc, s);
    return;
  }
  LOBPCG_ROCBLAS(rocblas_dgemm(h, ta, tb, m, n, k, &alpha, A, (rocblas_int)lda, B,
                               (rocblas_int)ldb, &beta, C, (rocblas_int)ldc));
}

void Dense::gemm(rocblas_operation ta, rocblas_operation tb, int m, int n, int k, double alpha,
                 const double* A, int64_t lda, const double* B, int64_t ldb, double beta,
                 double* C, int64_t ldc) {
  dgemm(h_, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc);
}

static void copy_cm(int m, int n, const double* src, int64_t lds, double* dst, int64_t ldd,
                    hipStream_t s);

void Dense::syev(int n, double* A, int64_t lda, double* w) {
  int32_t* dinfo = info_.as<int32_t>() + 2;
  if (n >= 2 && n <= kTridiagMaxN) {
    // Householder tridiagonalisation in one workgroup (kernels.hip), then
    // divide and conquer on the tridiagonal and the back-transformation Q Z_T.
    double* e = E_.as<double>();
    double* tau = tau_.as<double>();
    double* Z = T1_.as<double>();
    int tok = timer_ ? timer_->start(s_) : -1;
    launch_sytrd_lower(n, A, lda, w, e, tau, s_);
    if (timer_) {
      timer_->stop(tok, 5, 4.0 / 3.0 * n * (double)n * n, s_);
      tok = timer_->start(s_);
    }
    tridiag_dc(n, w, e, w, Z, nsmax_, Mt_.as<double>(), ZQ_.as<double>(), Qs_.as<double>(),
               dcY_.as<double>(), dcv_.as<double>(), dci_.as<int32_t>(), dcw_.as<double>(),
               dcr_.as<double>(), status_word(), h_, s_);
    if (timer_) {
      timer_->stop(tok, 6, 0.0, s_);
      tok = timer_->start(s_);
    }
    launch_ormtr_lower(n, A, lda, tau, Z, nsmax_, s_);
    if (timer_) timer_->stop(tok, 7, 0.0, s_);
    copy_cm(n, n, Z, nsmax_, A, lda, s_);
  } else {
    LOBPCG_ROCBLAS(rocsolver_dsyevd(h_, rocblas_evect_original, rocblas_fill_upper, n, A,
                                    (rocblas_int)lda, w, E_.as<double>(), dinfo));
  }
}

static void copy_cm(int m, int n, const double* src, int64_t lds, double* dst, int64_t ldd,
                    hipStream_t s) {
  if (m == 0 || n == 0) return;
  LOBPCG_HIP(hipMemcpy2DAsync(dst, sizeof(double) * ldd, src, sizeof(double) * lds,
                              sizeof(double) * m, n, hipMemcpyDeviceToDevice, s));
}

void Dense::join_p() {
  if (!p_pending_) return;
  LOBPCG_HIP(hipStreamWaitEvent(s_, ev_p_, 0));
  p_pending_ = false;
}

void Dense::extend_p() {
  if (p_pending_) LOBPCG_HIP(hipEventRecord(ev_p_, s2_));
}

// Mt = (Z_1(:, nc:nx)^T Z_1perp)^T = Z_1perp^T Z_1(:, nc:nx)   (m x na), or its
// literal reading (the first n_x - n_c rows of Z_1perp, transposed).
static void p_operand(const double* Z, int64_t ld, int ns, int nx, int nc, bool literal_lq,
                      double* Mt, int64_t ldm, rocblas_handle h) {
  const int m = ns - nx;
  const int na = nx - nc;
  if (literal_lq) {
    // Q_1perp rows from the LQ of Z_1perp; the first n_x - n_c of them span
    // the first n_x - n_c rows of Z_1perp: factor those rows only.
    const double one = 1.0, zero = 0.0;
    LOBPCG_ROCBLAS(rocblas_dgeam(h, rocblas_operation_transpose, rocblas_operation_none, m, na,
                                 &one, Z + nx * ld, (rocblas_int)ld, &zero, Mt, (rocblas_int)ldm,
                                 Mt, (rocblas_int)ldm));
  } else {
    dgemm(h, rocblas_operation_transpose, rocblas_operation_none, m, na, nx, 1.0, Z + nx * ld, ld,
          Z + nc * ld, ld, 0.0, Mt, ldm);
  }
}

void Dense::rr_p_block(const double* Z, int ns, int nx, int nc, bool literal_lq,
                       const double* theta, double* C, int64_t ldc, double* theta_p, int64_t ldtp,
                       hipStream_t s, rocblas_handle h) {
  const int64_t ld = nsmax_;
  const int m = ns - nx;
  const int na = nx - nc;
  const int np = std::min(na, m);
  const double* T = Ri_.as<double>();
  double* Mt = Mt_.as<double>();
  const int64_t ldm = ld;
  (void)literal_lq;
  // LQ of Mt^T == QR of Mt (Householder): Q (m x np) orthonormal columns.
  // Only the first np columns enter Q (np = min(na, m)).
  if (geqrf_orgqr_fits(m, np)) {
    const int tok = timer_ ? timer_->start(s) : -1;
    launch_geqrf_orgqr(m, np, Mt, ldm, s);
    if (timer_) timer_->stop(tok, 7, 0.0, s);
  } else {
    LOBPCG_ROCBLAS(rocsolver_dgeqrf(h, m, na, Mt, (rocblas_int)ldm, tau_.as<double>()));
    LOBPCG_ROCBLAS(rocsolver_dorgqr(h, m, np, np, Mt, (rocblas_int)ldm, tau_.as<double>()));
  }
  // C_p = T Z_perp Q.
  double* ZQ = ZQ_.as<double>();
  dgemm(h, rocblas_operation_none, rocblas_operation_none, ns, np, m, 1.0, Z + nx * ld, ld, Mt, ldm,
        0.0, ZQ, ld);
  dgemm(h, rocblas_operation_none, rocblas_operation_none, ns, np, ns, 1.0, T, ld, ZQ, ld, 0.0,
        C + nx * ldc, ldc);
  // Algorithm 7's Theta_p = Q^T Theta_perp Q.
  double* Qs = Qs_.as<double>();
  launch_row_scale_copy(m, np, theta + nx, Mt, ldm, Qs, ld, s);
  dgemm(h, rocblas_operation_transpose, rocblas_operation_none, np, np, m, 1.0, Mt, ldm, Qs, ld, 0.0,
        theta_p, ldtp);
  launch_symmetrize(np, theta_p, ldtp, s);
}

RROutput Dense::rr_modified(const double* GA, const double* GB, int64_t ldg, int ns, int nx,
                            int nc, bool use_ortho, bool literal_lq, double tau_skip, double* C,
                            int64_t ldc, double* theta, double* theta_p, int64_t ldtp,
                            bool defer_p, int n_ident, bool basic_p) {
  LOBPCG_CHECK(ns <= nsmax_ && nx <= ns && nc <= nx && n_ident >= 0 && n_ident <= ns,
               LOBPCG_ERR_ARG, "rr_modified: bad sizes");
  join_p();
  RROutput out;
  const int64_t ld = nsmax_;
  double* H = H_.as<double>();
  double* T = Ri_.as<double>();  // R^-1, then T = D R^-1 (or I)
  double* d = d_.as<double>();
  int32_t* dinfo = info_.as<int32_t>();
  if (!use_ortho) {
    double* R = R_.as<double>();
    // Algorithm 7's scaling and factor: D = diag(S^T B S)^-1/2, R^T R = D S^T B S D.
    launch_diag_scale(ns, GB, ldg, d, R, ld, true, s_);
    launch_diag_scale(ns, GA, ldg, d, H, ld, false, s_);
    const int k = n_ident, wn = ns - n_ident;
    int pivot_base = 0;
    if (k > 0 && wn > 0 && wn <= cholinv_max_n()) {
      // The leading k x k block of D S^T B S is exactly I (D is 1 there), so
      // with K its k x w upper-right block: R = [I K; 0 R_w] where R_w^T R_w =
      // G_w - K^T K, and R^-1 = [I, -K R_w^-1; 0, R_w^-1].  The lower-left
      // block of R keeps K^T: only R's upper triangle is read afterwards.
      double* K = R + (int64_t)k * ld;
      double* Rw = K + k;
      double* Tw = T + k + (int64_t)k * ld;
      gemm(rocblas_operation_transpose, rocblas_operation_none, wn, wn, k, -1.0, K, ld, K, ld,
           1.0, Rw, ld);
      const int tok = timer_ ? timer_->start(s_) : -1;
      launch_cholinv_upper(wn, Rw, ld, Tw, ld, dinfo, s_);
      if (timer_) timer_->stop(tok, 8, 2.0 / 3.0 * wn * (double)wn * wn, s_);
      launch_set_identity(ns, k, T, ld, s_);
      gemm(rocblas_operation_none, rocblas_operation_none, k, wn, wn, -1.0, K, ld, Tw, ld, 0.0,
           T + (int64_t)k * ld, ld);
      pivot_base = k;
    } else if (ns <= cholinv_max_n()) {
      // R and R^-1 from one sweep over [R^T R | I] in one workgroup.
      const int tok = timer_ ? timer_->start(s_) : -1;
      launch_cholinv_upper(ns, R, ld, T, ld, dinfo, s_);
      if (timer_) timer_->stop(tok, 8, 2.0 / 3.0 * ns * (double)ns * ns, s_);
    } else {
      LOBPCG_ROCBLAS(rocsolver_dpotrf(h_, rocblas_fill_upper, ns, R, (rocblas_int)ld, dinfo));
      launch_zero_lower(ns, R, ld, s_);
      copy_cm(ns, ns, R, ld, T, ld, s_);
      LOBPCG_ROCBLAS(rocsolver_dtrtri(h_, rocblas_fill_upper, rocblas_diagonal_non_unit, ns, T,
                                      (rocblas_int)ld, dinfo + 1));
      launch_zero_lower(ns, T, ld, s_);
    }
    launch_cond1_upper(ns, R, T, ld, cond_.as<double>(), E_.as<double>(), s_);
    LOBPCG_HIP(hipMemcpyAsync(hinfo_, dinfo, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s_));
    LOBPCG_HIP(hipMemcpyAsync(hcond_, cond_.get(), sizeof(double), hipMemcpyDeviceToHost, s_));
    LOBPCG_HIP(hipStreamSynchronize(s_));
    out.potrf_info = hinfo_[0] != 0 ? hinfo_[0] + pivot_base : 0;
    out.trtri_info = hinfo_[1];
    // a factorisation that broke down has no condition number (partial factors)
    out.cond = (hinfo_[0] != 0 || hinfo_[1] != 0) ? HUGE_VAL : hcond_[0];
    // Algorithm 7's rejection test (section 5.3 reading): cond(R)^3 tau_skip > 1.
    const bool bad_factor = hinfo_[0] != 0 || hinfo_[1] != 0 || !std::isfinite(out.cond);
    const bool ill = tau_skip > 0.0 && out.cond * out.cond * out.cond * tau_skip > 1.0;
    if (bad_factor || ill) {
      out.flipped = true;
      return out;
    }
    // The standard eigenproblem (R^-T D GA D R^-1) Z = Z Theta.
    double* T1 = T1_.as<double>();
    gemm(rocblas_operation_none, rocblas_operation_none, ns, ns, ns, 1.0, H, ld, T, ld, 0.0, T1,
         ld);
    gemm(rocblas_operation_transpose, rocblas_operation_none, ns, ns, ns, 1.0, T, ld, T1, ld, 0.0,
         H, ld);
    launch_symmetrize(ns, H, ld, s_);
    syev(ns, H, ld, theta);
    // T = D R^-1, the map from Z to coefficients of S.
    launch_row_scale(ns, ns, d, T, ld, s_);
  } else {
    // With useOrtho S is B-orthonormal: solve (S^T A S) Z = Z Theta directly.
    copy_cm(ns, ns, GA, ldg, H, ld, s_);
    launch_symmetrize(ns, H, ld, s_);
    syev(ns, H, ld, theta);
    launch_set_identity(ns, ns, T, ld, s_);
  }
  const double* Z = H;
  if (basic_p) {
    // C_x = T Z(:, 1:n_x); C_p = C_x with the rows of X zeroed
    gemm(rocblas_operation_none, rocblas_operation_none, ns, nx, ns, 1.0, T, ld, Z, ld, 0.0, C,
         ldc);
    LOBPCG_HIP(hipMemcpy2DAsync(C + (int64_t)nx * ldc, sizeof(double) * ldc, C,
                                sizeof(double) * ldc, sizeof(double) * ns, nx,
                                hipMemcpyDeviceToDevice, s_));
    LOBPCG_HIP(hipMemset2DAsync(C + (int64_t)nx * ldc, sizeof(double) * ldc, 0,
                                sizeof(double) * nx, nx, s_));
    out.np = nx;
    return out;
  }
  const int m = ns - nx;
  const int na = nx - nc;
  const int np = std::min(na, m);
  out.np = np;
  if (np > 0 && defer_p) {
    // The P block (LQ, C_p, Theta_p) on the second stream: the LQ operand is formed first, so that
    // the one-workgroup QR is queued before the main stream's next all-CU work.
    p_operand(Z, ld, ns, nx, nc, literal_lq, Mt_.as<double>(), ld, h_);
    LOBPCG_HIP(hipEventRecord(ev_z_, s_));
    LOBPCG_HIP(hipStreamWaitEvent(s2_, ev_z_, 0));
    rr_p_block(Z, ns, nx, nc, literal_lq, theta, C, ldc, theta_p, ldtp, s2_, h2_);
    LOBPCG_HIP(hipEventRecord(ev_p_, s2_));
    p_pending_ = true;
  }
  // C_x = T [Z_1; Z_2].
  gemm(rocblas_operation_none, rocblas_operation_none, ns, nx, ns, 1.0, T, ld, Z, ld, 0.0, C, ldc);
  if (np > 0 && !defer_p) {
    p_operand(Z, ld, ns, nx, nc, literal_lq, Mt_.as<double>(), ld, h_);
    rr_p_block(Z, ns, nx, nc, literal_lq, theta, C, ldc, theta_p, ldtp, s_, h_);
  }
  return out;
}

int Dense::svqb_transform(double* G, int64_t ldg, int nu, double tau, bool drop, double* Tu) {
  join_p();
  if (nu == 0) return 0;
  double* d = d_.as<double>();
  double* th = th2_.as<double>();
  double* sc = scale_.as<double>();
  int32_t* si = sinfo_.as<int32_t>();
  // D = diag(U^T M U)^-1/2; eig(D U^T M U D) = Z Theta.
  launch_diag_scale(nu, G, ldg, d, G, ldg, true, s_);
  syev(nu, G, ldg, th);
  launch_svqb_theta(nu, th, tau, drop ? 1 : 0, sc, si, s_);
  LOBPCG_HIP(hipMemcpyAsync(hinfo_ + 4, si, sizeof(int32_t) * 2, hipMemcpyDeviceToHost, s_));
  LOBPCG_HIP(hipStreamSynchronize(s_));
  const int first = hinfo_[4], keep = hinfo_[5];
  if (keep <= 0) return 0;
  // Tu = D Z(:, J) Theta(J)^-1/2
  launch_col_scale(nu, keep, G + (int64_t)first * ldg, ldg, sc + first, 0, Tu, nu, s_);
  launch_row_scale(nu, keep, d, Tu, nu, s_);
  return keep;
}

}  // namespace lobpcg
