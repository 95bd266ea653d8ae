// extern "C" boundary of the library (include/lobpcg.h, include/lobpcg_steps.h).
// Every entry point converts internal errors into status codes; nothing throws
// across the ABI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <exception>
#include <memory>
#include <new>
#include <string>

#include "common.hpp"
#include "dense.hpp"
#include "kernels.hpp"
#include "lobpcg.h"
#include "lobpcg_steps.h"
#include "hermitian.hpp"
#include "solver.hpp"

// A handle owns a real solver, or a complex Hermitian driver with its real
// solver inside; `solver` points at the real solver either way.
struct lobpcg_ctx {
  std::unique_ptr<lobpcg::Solver> own;
  std::unique_ptr<lobpcg::Hermitian> herm;
  lobpcg::Solver* solver = nullptr;
};

namespace {
thread_local std::string g_last_error;

template <typename F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const lobpcg::Error& e) {
    g_last_error = e.what();
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return LOBPCG_ERR_ALLOC;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return LOBPCG_ERR_HIP;
  } catch (...) {
    g_last_error = "unknown error";
    return LOBPCG_ERR_HIP;
  }
}

hipStream_t as_stream(void* s) { return static_cast<hipStream_t>(s); }
}  // namespace

extern "C" {

void lobpcg_default_options(lobpcg_options* opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->block_size = 0;
  opt->maxit = 2000;
  opt->precision = 0;
  opt->precond = 0;
  opt->implicit_products = -1;
  opt->lq_literal = 0;
  opt->tau_ortho = 1e-12;
  opt->drop_factor = 10.0;
  opt->replace_factor = 10.0;
  opt->skip_factor = 10.0;
  opt->fp32_tol = 1e-5;
  opt->seed = 0;
  opt->stream = nullptr;
  opt->ortho_mode = 0;
  opt->force_ortho = 0;
  opt->implicit_gram = 1;
  opt->basic = 0;
  opt->largest = 0;
}

int lobpcg_create(lobpcg_t* out, const lobpcg_csr* A, const lobpcg_csr* B, int32_t k,
                  const lobpcg_options* opt) {
  return guarded([&]() {
    LOBPCG_CHECK(out != nullptr, LOBPCG_ERR_ARG, "out is NULL");
    *out = nullptr;
    lobpcg_options o;
    if (opt) o = *opt;
    else lobpcg_default_options(&o);
    std::unique_ptr<lobpcg_ctx> h(new lobpcg_ctx);
    h->own.reset(new lobpcg::Solver(A, B, k, o));
    h->solver = h->own.get();
    *out = h.release();
    return LOBPCG_OK;
  });
}

int lobpcg_create_hermitian(lobpcg_t* out, const lobpcg_zcsr* A, const lobpcg_zcsr* B, int32_t k,
                            const lobpcg_options* opt) {
  return guarded([&]() {
    LOBPCG_CHECK(out != nullptr, LOBPCG_ERR_ARG, "out is NULL");
    *out = nullptr;
    lobpcg_options o;
    if (opt) o = *opt;
    else lobpcg_default_options(&o);
    std::unique_ptr<lobpcg_ctx> h(new lobpcg_ctx);
    h->herm.reset(new lobpcg::Hermitian(A, B, k, o));
    h->solver = &h->herm->real();
    *out = h.release();
    return LOBPCG_OK;
  });
}

int lobpcg_solve_hermitian(lobpcg_t h, double tol, const double* X0_re, const double* X0_im,
                           int32_t x0_on_device, lobpcg_precond_fn K, void* K_user,
                           lobpcg_info* info) {
  return guarded([&]() {
    LOBPCG_CHECK(h && h->herm, LOBPCG_ERR_ARG, "not a complex Hermitian handle");
    return h->herm->solve(tol, X0_re, X0_im, x0_on_device != 0, K, K_user, info);
  });
}

int lobpcg_eigpairs_hermitian(lobpcg_t h, int32_t count, double* lambda, double* X_re,
                              double* X_im, int64_t ldx, double* rel_resid, int32_t on_device) {
  return guarded([&]() {
    LOBPCG_CHECK(h && h->herm, LOBPCG_ERR_ARG, "not a complex Hermitian handle");
    return h->herm->eigpairs(count, lambda, X_re, X_im, ldx, rel_resid, on_device != 0);
  });
}

int lobpcg_solve(lobpcg_t h, double tol, const double* X0, int32_t x0_on_device,
                 lobpcg_precond_fn K, void* K_user, lobpcg_info* info) {
  return guarded([&]() {
    LOBPCG_CHECK(h && h->solver, LOBPCG_ERR_ARG, "NULL handle");
    LOBPCG_CHECK(!h->herm, LOBPCG_ERR_ARG, "complex Hermitian handle: use the _hermitian calls");
    return h->solver->solve(tol, X0, x0_on_device != 0, K, K_user, info);
  });
}

int lobpcg_eigpairs(lobpcg_t h, int32_t count, double* lambda, double* X, int64_t ldx,
                    double* rel_resid, int32_t on_device) {
  return guarded([&]() {
    LOBPCG_CHECK(h && h->solver, LOBPCG_ERR_ARG, "NULL handle");
    LOBPCG_CHECK(!h->herm, LOBPCG_ERR_ARG, "complex Hermitian handle: use the _hermitian calls");
    return h->solver->eigpairs(count, lambda, X, ldx, rel_resid, on_device != 0);
  });
}

int lobpcg_adjoint(lobpcg_t h, int32_t count, const double* lambda_bar, const double* X_bar,
                   int64_t ld_xbar, double* grad, double* grad_B, double cg_tol,
                   int32_t cg_maxit, int32_t* cg_iters) {
  return guarded([&]() {
    LOBPCG_CHECK(h && h->solver, LOBPCG_ERR_ARG, "NULL handle");
    LOBPCG_CHECK(!h->herm, LOBPCG_ERR_ARG, "complex Hermitian handle: use the _hermitian calls");
    return h->solver->adjoint(count, lambda_bar, X_bar, ld_xbar, grad, grad_B, cg_tol, cg_maxit,
                              cg_iters);
  });
}

int lobpcg_dims(lobpcg_t h, int64_t* n, int32_t* k, int32_t* n_x) {
  return guarded([&]() {
    LOBPCG_CHECK(h && h->solver, LOBPCG_ERR_ARG, "NULL handle");
    if (h->herm) {
      if (n) *n = h->herm->n();
      if (k) *k = h->herm->k();
      if (n_x) *n_x = h->herm->nx();
      return LOBPCG_OK;
    }
    if (n) *n = h->solver->n();
    if (k) *k = h->solver->k();
    if (n_x) *n_x = h->solver->nx();
    return LOBPCG_OK;
  });
}

void lobpcg_destroy(lobpcg_t h) {
  try {
    delete h;
  } catch (...) {
  }
}

const char* lobpcg_last_error(void) { return g_last_error.c_str(); }

int lobpcg_kernel_stats(lobpcg_t h, int32_t enable, lobpcg_kernel_stat* out) {
  return guarded([&]() {
    LOBPCG_CHECK(h && h->solver, LOBPCG_ERR_ARG, "NULL handle");
    lobpcg::KernelTimer& t = h->solver->timer();
    t.collect();
    if (out)
      for (int i = 0; i < LOBPCG_KERNEL_KINDS; ++i) out[i] = t.totals[i];
    t.enable(enable != 0);
    return LOBPCG_OK;
  });
}

int lobpcg_set_profiling(lobpcg_t h, int32_t on) {
  return guarded([&]() {
    LOBPCG_CHECK(h && h->solver, LOBPCG_ERR_ARG, "NULL handle");
    h->solver->set_profiling(on != 0);
    return LOBPCG_OK;
  });
}

// ------------------------------------------------------------------ steps
int lobpcg_spmm(int64_t n, const int64_t* rowptr, const int32_t* colind, const void* values,
                int32_t dtype, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t ncols,
                void* stream) {
  return guarded([&]() {
    LOBPCG_CHECK(n >= 0 && ncols >= 0 && ldx >= ncols && ldy >= ncols, LOBPCG_ERR_ARG,
                 "lobpcg_spmm: bad sizes");
    LOBPCG_CHECK(dtype == 0 || dtype == 1, LOBPCG_ERR_ARG, "dtype must be 0 or 1");
    if (dtype == 0)
      lobpcg::launch_spmm<double>(n, rowptr, colind, (const double*)values, (const double*)X, ldx,
                                  (double*)Y, ldy, ncols, as_stream(stream));
    else
      lobpcg::launch_spmm<float>(n, rowptr, colind, (const float*)values, (const float*)X, ldx,
                                 (float*)Y, ldy, ncols, as_stream(stream));
    return LOBPCG_OK;
  });
}

int64_t lobpcg_gram_workspace(int64_t n, int32_t m, int32_t p, int32_t dtype) {
  if (n < 0 || m < 0 || p < 0 || (dtype != 0 && dtype != 1)) return -1;
  return lobpcg::gram_workspace_bytes(n, m, p, dtype == 1);
}

int lobpcg_gram(int64_t n, int32_t m, int32_t p, int32_t p1, int32_t dtype, const void* L,
                int64_t ldl, const void* R1, int64_t ldr1, const void* R2, int64_t ldr2,
                double* G, int64_t ldg, int32_t col_offset, int32_t mirror, void* work,
                void* stream) {
  return guarded([&]() {
    LOBPCG_CHECK(n >= 0 && m >= 0 && p >= 0 && p1 >= 0 && p1 <= p && ldl >= m && ldg >= m &&
                     col_offset >= 0,
                 LOBPCG_ERR_ARG, "lobpcg_gram: bad sizes");
    LOBPCG_CHECK(p1 == p || R2 != nullptr, LOBPCG_ERR_ARG, "lobpcg_gram: R2 missing");
    LOBPCG_CHECK(dtype == 0 || dtype == 1, LOBPCG_ERR_ARG, "dtype must be 0 or 1");
    LOBPCG_CHECK(!mirror || (col_offset <= m && ldg >= col_offset + p), LOBPCG_ERR_ARG,
                 "lobpcg_gram: mirror needs col_offset <= m and ldg >= col_offset + p");
    const int mr = mirror ? std::min<int32_t>(col_offset, m) : 0;
    if (dtype == 0)
      lobpcg::launch_gram<double>(n, m, p, p1, (const double*)L, ldl, (const double*)R1, ldr1,
                                  (const double*)R2, ldr2, G, col_offset, G, col_offset + p1, ldg,
                                  mr, work, as_stream(stream));
    else
      lobpcg::launch_gram<float>(n, m, p, p1, (const float*)L, ldl, (const float*)R1, ldr1,
                                 (const float*)R2, ldr2, G, col_offset, G, col_offset + p1, ldg,
                                 mr, work, as_stream(stream));
    return LOBPCG_OK;
  });
}

int lobpcg_gram_noalloc(int64_t n, int32_t m, int32_t p, int32_t p1, int32_t dtype,
                        const void* L, int64_t ldl, const void* R1, int64_t ldr1, const void* R2,
                        int64_t ldr2, double* G, int64_t ldg, int32_t col_offset, int32_t mirror,
                        void* stream) {
  return guarded([&]() {
    LOBPCG_CHECK(n >= 0 && m >= 0 && p >= 0 && p1 >= 0 && p1 <= p && ldl >= m && ldg >= m &&
                     col_offset >= 0,
                 LOBPCG_ERR_ARG, "lobpcg_gram_noalloc: bad sizes");
    LOBPCG_CHECK(p1 == p || R2 != nullptr, LOBPCG_ERR_ARG, "lobpcg_gram_noalloc: R2 missing");
    LOBPCG_CHECK(dtype == 0 || dtype == 1, LOBPCG_ERR_ARG, "dtype must be 0 or 1");
    LOBPCG_CHECK(!mirror || (col_offset <= m && ldg >= col_offset + p), LOBPCG_ERR_ARG,
                 "lobpcg_gram_noalloc: mirror needs col_offset <= m and ldg >= col_offset + p");
    const int mr = mirror ? std::min<int32_t>(col_offset, m) : 0;
    if (dtype == 0)
      lobpcg::launch_gram_noalloc<double>(n, m, p, p1, (const double*)L, ldl, (const double*)R1,
                                          ldr1, (const double*)R2, ldr2, G, col_offset, G,
                                          col_offset + p1, ldg, mr, as_stream(stream));
    else
      lobpcg::launch_gram_noalloc<float>(n, m, p, p1, (const float*)L, ldl, (const float*)R1,
                                         ldr1, (const float*)R2, ldr2, G, col_offset, G,
                                         col_offset + p1, ldg, mr, as_stream(stream));
    return LOBPCG_OK;
  });
}

int64_t lobpcg_gram_noalloc_max_bytes(void) { return lobpcg::kGramScratchBytes; }

int lobpcg_update(int64_t n, int32_t K, int32_t N, int32_t dtype, const void* S, int64_t lds,
                  const double* C, int64_t ldc, double alpha, double beta, void* Y, int64_t ldy,
                  void* stream) {
  return guarded([&]() {
    LOBPCG_CHECK(n >= 0 && K >= 0 && N >= 0 && lds >= K && ldc >= K && ldy >= N, LOBPCG_ERR_ARG,
                 "lobpcg_update: bad sizes");
    LOBPCG_CHECK(beta == 0.0 || beta == 1.0, LOBPCG_ERR_ARG, "beta must be 0 or 1");
    if (dtype == 0)
      lobpcg::launch_update<double>(n, K, N, (const double*)S, lds, C, ldc, alpha, beta,
                                    (double*)Y, ldy, as_stream(stream));
    else
      lobpcg::launch_update<float>(n, K, N, (const float*)S, lds, C, ldc, alpha, beta, (float*)Y,
                                   ldy, as_stream(stream));
    return LOBPCG_OK;
  });
}

int64_t lobpcg_residual_workspace(int64_t n, int32_t nx) {
  if (n < 0 || nx < 0) return -1;
  return lobpcg::residual_workspace_bytes(n, nx);
}

int lobpcg_residual(int64_t n, int32_t nx, int32_t dtype, const void* AX, int64_t ldax,
                    const void* BX, int64_t ldbx, const void* X, int64_t ldx,
                    const double* theta, const double* dinv, void* W, int64_t ldw, double normA,
                    double normB, double tol, double* rho, int32_t* n_c_out, void* work,
                    void* stream) {
  return guarded([&]() {
    LOBPCG_CHECK(n >= 0 && nx >= 0 && ldax >= nx && ldx >= nx && (!W || ldw >= nx) &&
                     (!BX || ldbx >= nx),
                 LOBPCG_ERR_ARG, "lobpcg_residual: bad sizes");
    if (dtype == 0)
      lobpcg::launch_residual<double>(n, nx, (const double*)AX, ldax, (const double*)BX, ldbx,
                                      (const double*)X, ldx, theta, dinv, (double*)W, ldw, normA,
                                      normB, tol, rho, n_c_out, work, as_stream(stream));
    else
      lobpcg::launch_residual<float>(n, nx, (const float*)AX, ldax, (const float*)BX, ldbx,
                                     (const float*)X, ldx, theta, dinv, (float*)W, ldw, normA,
                                     normB, tol, rho, n_c_out, work, as_stream(stream));
    return LOBPCG_OK;
  });
}

int64_t lobpcg_spmm_residual_workspace(int64_t n, int32_t nx) {
  if (n < 0 || nx < 0) return -1;
  return lobpcg::spmm_residual_workspace_bytes(n, nx);
}

int lobpcg_spmm_residual(int64_t n, const int64_t* rowptr, const int32_t* colind,
                         const void* values, int32_t dtype, const void* X, int64_t ldx,
                         int32_t nx, const double* theta, const double* dinv, void* W,
                         int64_t ldw, void* AX, int64_t ldax, double normA, double tol,
                         double* rho, int32_t* n_c_out, void* work, void* stream) {
  return guarded([&]() {
    LOBPCG_CHECK(n >= 0 && nx >= 0 && ldx >= nx && W && ldw >= nx && (!AX || ldax >= nx) &&
                     (dtype == 0 || dtype == 1),
                 LOBPCG_ERR_ARG, "lobpcg_spmm_residual: bad arguments");
    if (dtype == 0)
      lobpcg::launch_spmm_residual<double>(n, rowptr, colind, (const double*)values,
                                           (const double*)X, ldx, nx, theta, dinv, (double*)W,
                                           ldw, (double*)AX, ldax, normA, tol, rho, n_c_out,
                                           work, as_stream(stream));
    else
      lobpcg::launch_spmm_residual<float>(n, rowptr, colind, (const float*)values,
                                          (const float*)X, ldx, nx, theta, dinv, (float*)W, ldw,
                                          (float*)AX, ldax, normA, tol, rho, n_c_out, work,
                                          as_stream(stream));
    return LOBPCG_OK;
  });
}

int lobpcg_rr_step(int32_t n_s, int32_t n_x, int32_t n_c, int32_t use_ortho, int32_t lq_literal,
                   int32_t n_ident, const double* GA, const double* GB, int64_t ldg,
                   double tau_skip, double* C,
                   int64_t ldc, double* theta, double* theta_p, int32_t* n_p, int32_t* flipped,
                   double* cond, void* stream) {
  return guarded([&]() {
    LOBPCG_CHECK(n_s >= 1 && n_x >= 1 && n_x <= n_s && n_c >= 0 && n_c <= n_x && ldg >= n_s &&
                     ldc >= n_s && n_ident >= 0 && n_ident <= n_s,
                 LOBPCG_ERR_ARG, "lobpcg_rr_step: bad sizes");
    lobpcg::Dense d(n_s, n_x, as_stream(stream));
    lobpcg::RROutput o = d.rr_modified(GA, GB, ldg, n_s, n_x, n_c, use_ortho != 0,
                                       lq_literal != 0, tau_skip, C, ldc, theta, theta_p, n_x,
                                       false, n_ident);
    int32_t stalled = 0;
    LOBPCG_HIP(hipMemcpyAsync(&stalled, d.status_word(), sizeof(int32_t), hipMemcpyDeviceToHost,
                              as_stream(stream)));
    LOBPCG_HIP(hipStreamSynchronize(as_stream(stream)));
    LOBPCG_CHECK(stalled != 2, LOBPCG_ERR_NONFINITE, "non-finite projected matrix");
    LOBPCG_CHECK(stalled == 0, LOBPCG_ERR_BREAKDOWN,
                 "projected eigenproblem: an implicit QL leaf did not converge");
    if (n_p) *n_p = o.np;
    if (flipped) *flipped = o.flipped ? 1 : 0;
    if (cond) *cond = o.cond;
    return LOBPCG_OK;
  });
}

}  // extern "C"
