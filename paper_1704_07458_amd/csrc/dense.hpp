// FP64 dense routines on the device for the projected problems of the
// robust LOBPCG: Rayleigh-Ritz with improved basis selection (Algorithm 7,
// also used for Algorithm 2 on the initial block) and the small eigenproblems
// of SVQB (Algorithms 4 and 6).  Built on rocSOLVER / rocBLAS (column-major)
// plus the small kernels of kernels.hip.
#pragma once

#include <rocblas/rocblas.h>

#include <cstdint>

#include "common.hpp"
#include "timer.hpp"

namespace lobpcg {

struct RROutput {
  int np = 0;           // columns of C_p
  bool flipped = false; // Cholesky rejected (section 5.3): no coefficients
  double cond = 0.0;    // cond_1 of the scaled Cholesky factor (0 when unused)
  int potrf_info = 0, trtri_info = 0;
};

class Dense {
 public:
  // nsmax: largest projected dimension; nxmax: largest n_x.
  Dense(int nsmax, int nxmax, hipStream_t s);
  ~Dense();
  Dense(const Dense&) = delete;
  Dense& operator=(const Dense&) = delete;

  // Algorithm 7 on (GA, GB) (column-major, ldg).  Writes C = [C_x, C_p]
  // (ns x (nx + np), column-major, ldc), theta (ns, ascending) and theta_p
  // (np x np, column-major, ld ldtp).  GB is unused when use_ortho.  tau_skip <= 0
  // disables the conditioning test (Algorithm 2).  Synchronises the stream once
  // (to read the Cholesky status and cond) unless use_ortho.
  //
  // defer_p: the P block (the QR of Alg. 7's LQ operand, C_p, Theta_p) is left
  // running on the second stream; C_x is complete on the main stream when the
  // call returns, C_p and Theta_p only after join_p().
  //
  // n_ident: the leading n_ident x n_ident block of GB is exactly the identity
  // (the X and P blocks of eqs. (12)-(14)); the Cholesky factor is then formed
  // blockwise and only the Schur complement of the W block is factored.
  //
  // basic_p: Algorithm 1's P instead of the P block of Algorithm 7:
  // C_p = C_x with its first n_x rows zeroed (P = S(:, n_x+1:end) C(n_x+1:end, 1:n_x)), n_p = n_x.
  RROutput rr_modified(const double* GA, const double* GB, int64_t ldg, int ns, int nx, int nc,
                       bool use_ortho, bool literal_lq, double tau_skip, double* C, int64_t ldc,
                       double* theta, double* theta_p, int64_t ldtp, bool defer_p = false,
                       int n_ident = 0, bool basic_p = false);

  // Orders the main stream after the deferred P block (no-op when none).
  void join_p();
  // The deferred P block's stream, while one is pending (else nullptr): work
  // queued there follows the P block, and extend_p() makes join_p() wait for
  // it too.
  hipStream_t p_stream() const { return p_pending_ ? s2_ : nullptr; }
  void extend_p();

  // SVQB transform of Algorithms 4 / 6 from the Gram matrix G = U^T M U (nu x nu,
  // column-major, ldg; overwritten): Tu = D Z(:, J) Theta(J)^-1/2 written to Tu
  // (nu x nkeep, column-major, ld nu).  drop = false floors theta at tau*max|theta|
  // (keeps all); drop = true keeps theta_j > tau*max|theta|.  Returns nkeep
  // (synchronises the stream).
  int svqb_transform(double* G, int64_t ldg, int nu, double tau, bool drop, double* Tu);

  rocblas_handle handle() const { return h_; }
  // Grow the main handle's library workspace to at least `bytes` (from the
  // current allocator); callers size it with a device-memory size query.
  void reserve_library_workspace(size_t bytes);
  hipStream_t stream() const { return s_; }

  // Device status word that the tridiagonal eigensolver sets to 1 when an
  // implicit-QL leaf fails to converge (never cleared here; zero before use).
  // Default: a word of this object, zeroed at construction.
  int32_t* status_word() const { return status_ ? status_ : info_.as<int32_t>() + 7; }
  void set_status_word(int32_t* w) { status_ = w; }

  // Kernel-class timing of the tridiagonalisation (kind 5), the tridiagonal
  // eigensolver (kind 6) and the QR / back-transformation kernels (kind 7).
  void set_timer(KernelTimer* t) { timer_ = t; }

 private:
  void gemm(rocblas_operation ta, rocblas_operation tb, int m, int n, int k, double alpha,
            const double* A, int64_t lda, const double* B, int64_t ldb, double beta, double* C,
            int64_t ldc);
  // Eigenpairs of a symmetric n x n matrix (column-major, lda), ascending:
  // the one-workgroup tridiagonalisation, divide and conquer and
  // back-transformation for 2 <= n <= kTridiagMaxN, rocSOLVER's syevd otherwise.
  void syev(int n, double* A, int64_t lda, double* w);
  size_t library_workspace_bytes(rocblas_handle h);
  // Algorithm 7's P block (from Z and T = D R^-1 in place) on stream s with handle h.
  void rr_p_block(const double* Z, int ns, int nx, int nc, bool literal_lq, const double* theta,
                  double* C, int64_t ldc, double* theta_p, int64_t ldtp, hipStream_t s,
                  rocblas_handle h);

  int nsmax_, nxmax_;
  hipStream_t s_;
  rocblas_handle h_ = nullptr;
  // second stream (default priority) for Algorithm 7's P block (a
  // one-workgroup QR and small products) beside the main stream's all-CU
  // work, with its own rocBLAS handle
  hipStream_t s2_ = nullptr;
  rocblas_handle h2_ = nullptr;
  hipEvent_t ev_z_ = nullptr, ev_p_ = nullptr;
  bool p_pending_ = false;
  KernelTimer* timer_ = nullptr;
  int32_t* status_ = nullptr;
  int kTridiagMaxN = 512;
  // scratch (column-major, leading dimension nsmax_)
  DevBuf H_, R_, Ri_, T1_, Mt_, ZQ_, Qs_, d_, E_, tau_, info_, cond_, th2_, scale_, sinfo_;
  DevBuf dcY_, dcv_, dci_, dcw_, dcr_;  // divide-and-conquer workspace
  DevBuf lib_ws_, lib_ws2_;  // rocBLAS / rocSOLVER device workspace of h_ and h2_
  int32_t* hinfo_ = nullptr;  // pinned host status words
  double* hcond_ = nullptr;
};

}  // namespace lobpcg
