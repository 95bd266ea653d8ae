// Complex Hermitian pencils through the real embedding.
//
// The paper states Algorithms 2-8 for real pencils and notes that they carry
// over to complex Hermitian ones with conjugate transposes (section 1).  For
// A = Ar + i Ai Hermitian and x = xr + i xi, the real symmetric matrix
//   Ahat = [Ar  -Ai]
//          [Ai   Ar]
// maps the stacked vector [xr; xi] to the stacked A x, and the stacked
// vectors of x and i x, [xr; xi] and [-xi; xr], span a real two-dimensional
// space that Ahat keeps invariant (likewise for B).  Algorithm 8 on (Ahat,
// Bhat) started from the paired block [X0, i X0] therefore spans at every
// step the real form of the complex iteration's span (in exact arithmetic):
// its Ritz values are the complex ones, each twice.  The 2k smallest real
// Ritz pairs give the k smallest complex pairs: the complex vectors
// z_j = x_j(1:n) + i x_j(n+1:2n) of the 2k real Ritz vectors span the
// complex invariant subspace (rank k); its B-orthonormal basis Q comes from
// the k-dimensional range of Z^H B Z, and a complex Rayleigh-Ritz step on Q
// gives the eigenpairs.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>

#include "common.hpp"
#include "lobpcg.h"
#include "solver.hpp"

typedef struct _rocblas_handle* rocblas_handle;

namespace lobpcg {

class Hermitian {
 public:
  Hermitian(const lobpcg_zcsr* A, const lobpcg_zcsr* B, int k, const lobpcg_options& opt);
  ~Hermitian();

  int solve(double tol, const double* X0re, const double* X0im, bool x0_dev,
            lobpcg_precond_fn K, void* Kuser, lobpcg_info* info);
  int eigpairs(int count, double* lambda, double* Xre, double* Xim, int64_t ldx, double* rho,
               bool on_device);

  Solver& real() { return *solver_; }
  int64_t n() const { return n_; }
  int k() const { return k_; }
  int nx() const { return nx_; }

 private:
  void extract();
  void library_workspace();

  std::unique_ptr<Solver> solver_;
  int64_t n_ = 0;
  int k_ = 0, nx_ = 0;
  uint64_t seed_ = 0;
  rocblas_handle h_ = nullptr;
  bool extracted_ = false;
  // extraction buffers (complex values as interleaved pairs of doubles)
  DevBuf Xr_;     // 2n x 2k real Ritz vectors, row-major
  DevBuf Y_;      // 2n x max(2k, n_x) real scratch, row-major
  DevBuf Z_, BZ_, Q_, BQ_, AQ_;  // n x 2k / n x k complex, column-major
  DevBuf M_, V_;  // 2k x 2k complex
  DevBuf mu_, e_; // 2k reals
  DevBuf theta_, rho_;  // k reals
  DevBuf info_;
  DevBuf lib_ws_;
};

}  // namespace lobpcg
