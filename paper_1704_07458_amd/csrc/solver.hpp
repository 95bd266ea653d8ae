// Algorithm 8 (robust LOBPCG) driver on one GPU.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <string>
#include <vector>

#include "common.hpp"
#include "dense.hpp"
#include "lobpcg.h"

namespace lobpcg {

// Device copy of a CSR matrix (FP64 values, plus an FP32 copy for split mode).
struct DevCsr {
  int64_t n = 0, nnz = 0;
  DevBuf rowptr, colind, v64, v32;
};

// Per-precision block storage.  Every block is row-major with leading
// dimension ldS (= 3 n_x rounded up) or ldX (= n_x rounded up).
template <typename T>
struct Blocks {
  DevBuf S[2];  // [X | P | W], ping-pong
  DevBuf AX, AW, BXP, BW, MU, U2, R;
  DevBuf AS[2];  // [A X | A P | A W] in the layout of S (implicit product updates only)
  void alloc(int64_t n, int64_t ldS, int64_t ldX, bool haveB, bool implicit_products);
};


class Solver {
 public:
  Solver(const lobpcg_csr* A, const lobpcg_csr* B, int k, const lobpcg_options& opt);
  ~Solver();

  int solve(double tol, const double* X0, bool x0_dev, lobpcg_precond_fn K, void* Kuser,
            lobpcg_info* info);
  int eigpairs(int count, double* lambda, double* X, int64_t ldx, double* rho, bool on_device);
  int adjoint(int count, const double* lambda_bar, const double* X_bar, int64_t ld_xbar,
              double* grad, double* grad_B, double cg_tol, int cg_maxit, int32_t* cg_iters);
  bool has_B() const { return haveB_; }
  int64_t nnz_B() const { return haveB_ ? B_.nnz : 0; }

  int64_t n() const { return n_; }
  int k() const { return k_; }
  int nx() const { return nx_; }
  // For drivers built on this solver (the complex Hermitian embedding): the
  // stream, the allocator, the sketch norms and the stored operators.
  hipStream_t stream() const { return s_; }
  const DevAllocator* allocator() const { return &alloc_; }
  bool solved() const { return solved_; }
  bool largest() const { return opt_.largest != 0; }
  double norm_A_est() const { return normA_; }
  double norm_B_est() const { return normB_; }
  // Y = M X in FP64 on the solver's stream (M = A as stored, negated when
  // largest, or B; B = I copies X); row-major blocks with ncols columns.
  void apply(bool use_B, const double* X, int64_t ldx, double* Y, int64_t ldy, int ncols);
  void set_profiling(bool on) { profile_ = on; }
  KernelTimer& timer() { return timer_; }

 private:
  template <typename T>
  int run(Blocks<T>& b, const DevCsr& A, const DevCsr* B, double tol, int maxit,
          const double* X0dev, double tau_skip, double tau_ortho, lobpcg_precond_fn K,
          void* Kuser, lobpcg_info* info, int* iters_out);

  template <typename T>
  int ortho_drop(Blocks<T>& b, const DevCsr* B, T* U, int64_t ldu, int nu, const T* V,
                 int64_t ldv, const T* MV, int64_t ldmv, int nv, double tau_ortho, double eps,
                 lobpcg_info* info);

  template <typename T>
  void spmm(const DevCsr& M, const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols);

  template <typename T>
  void gram(int64_t n, int m, int p, int p1, const T* L, int64_t ldl, const T* R1, int64_t ldr1,
            const T* R2, int64_t ldr2, double* G1, int c1, double* G2, int c2, int64_t ldg,
            int mirror_rows);
  template <typename T>
  void update(int64_t n, int K, int N, const T* S, int64_t lds, const double* C, int64_t ldc,
              double alpha, double beta, T* Y, int64_t ldy, hipStream_t stream = nullptr);
  void phase_mark(int phase);
  void sync();
  // ||A||^(Omega), ||B||^(Omega) of section 4.3 from the seeded sketch.
  void sketch_norms();

  DevAllocator alloc_{};  // the caller's device-allocation hooks (or hipMalloc)
  hipStream_t s_ = nullptr;
  int64_t n_ = 0;
  int k_ = 0, nx_ = 0, nsmax_ = 0;
  int64_t ldS_ = 0, ldX_ = 0;
  lobpcg_options opt_{};
  DevCsr A_, B_;
  bool haveB_ = false;
  std::unique_ptr<Dense> dense_;
  Blocks<double> b64_;
  Blocks<float> b32_;
  DevBuf GA_, GB_, C_, theta_, theta_p_, rho_, dinv_, nc_, work_, X0buf_, nrm_;
  DevBuf C32_;  // FP32 copy of C for the library GEMM of the FP32 phase
  int32_t* hbuf_ = nullptr;   // pinned host words
  hipEvent_t ev_nc_ = nullptr;  // n_c copied to hbuf_ (the host waits for it alone)
  double* hdbl_ = nullptr;    // pinned host doubles
  // results
  bool solved_ = false;
  int final_nc_ = 0;
  double normA_ = 0.0, normB_ = 1.0;
  const double* Xres_ = nullptr;  // points into b64_.S[cur]
  bool profile_ = false;
  // FP32 phase of the precision split: a breakdown or non-finite value hands
  // over to the FP64 phase instead of ending the solve
  bool fp32_soft_ = false;
  bool fp32_stalled_ = false;
  static constexpr int kFp32StallIters = 200;
  std::string fp32_failure_;
  double tmark_ = 0.0;
  int cur_phase_ = 7;
  double* phase_acc_ = nullptr;
  KernelTimer timer_;
};

}  // namespace lobpcg
