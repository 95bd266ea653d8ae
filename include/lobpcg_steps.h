/*
 * lobpcg_steps.h -- the individual steps of one robust LOBPCG iteration
 * (arXiv 1704.07458, Algorithm 8) as separate C entry points.
 *
 * These are the same kernels lobpcg_solve() runs, exposed so that each step can
 * be checked on its own.  All pointers are DEVICE pointers unless stated;
 * dense blocks are row-major with the given leading dimension (in elements);
 * dtype 0 = double, 1 = float.  Work is enqueued on `stream` (hipStream_t,
 * NULL = default) and the call returns without synchronising unless stated.
 * Return codes are those of lobpcg.h.  Workspaces are caller-owned device
 * memory of at least the size reported by the matching *_workspace call.
 */
#ifndef LOBPCG_MI355X_STEPS_H
#define LOBPCG_MI355X_STEPS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Sparse times block, Y = A X (section 2 / Algorithm 8's residual and the products
 * A W, B W of section 5.2).  CSR as in lobpcg.h with values of type dtype; X is
 * n x ncols (ldx), Y is n x ncols (ldy), Y must not alias X.  ncols may be 0. */
int lobpcg_spmm(int64_t n, const int64_t* rowptr, const int32_t* colind, const void* values,
                int32_t dtype, const void* X, int64_t ldx, void* Y, int64_t ldy, int32_t ncols,
                void* stream);

/* Bytes of workspace lobpcg_gram needs for an (m x p) product over n rows. */
int64_t lobpcg_gram_workspace(int64_t n, int32_t m, int32_t p, int32_t dtype);

/* Block inner products G = L^T R (the Gram blocks S^T A W, S^T B W of
 * section 5.2; eqs. 12-14 give the rest).  L: n x m (ldl), R: n x p given as
 * two column segments R1 (n x p1, ldr1) and R2 (n x (p - p1), ldr2; may be NULL
 * when p1 = p).  Split-K over rows on MFMA with a deterministic second-stage
 * sum in FP64.  Output COLUMN-major FP64 with leading dimension ldg:
 * G(i, col_offset + j) = (L^T R)(i, j).  If mirror != 0 the rows i < col_offset
 * are also written transposed, G(col_offset + j, i), which completes a
 * symmetric m x m matrix whose last p = m - col_offset columns are computed
 * (the W columns of S^T A S); the written positions never overlap.
 * work: lobpcg_gram_workspace(n, m, p, dtype) bytes. */
int lobpcg_gram(int64_t n, int32_t m, int32_t p, int32_t p1, int32_t dtype, const void* L,
                int64_t ldl, const void* R1, int64_t ldr1, const void* R2, int64_t ldr2,
                double* G, int64_t ldg, int32_t col_offset, int32_t mirror, void* work,
                void* stream);

/* lobpcg_gram without a workspace, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same G, with the split-K partial tiles kept in a fixed
 * device array of lobpcg_gram_noalloc_max_bytes() bytes (16 MiB) that the
 * library holds on each GPU it runs on until the process ends (the split count
 * is reduced to fit, so the summation order may differ from lobpcg_gram within
 * the same rounding bound).  Nothing is allocated and no memset is issued.
 * Returns LOBPCG_ERR_ARG when m * p * 8 exceeds that size.  Every call on a
 * GPU shares that GPU's array: calls that overlap on one GPU (concurrent
 * streams or threads) race and must be serialised by the caller. */
int lobpcg_gram_noalloc(int64_t n, int32_t m, int32_t p, int32_t p1, int32_t dtype,
                        const void* L, int64_t ldl, const void* R1, int64_t ldr1, const void* R2,
                        int64_t ldr2, double* G, int64_t ldg, int32_t col_offset, int32_t mirror,
                        void* stream);

/* Size in bytes of lobpcg_gram_noalloc's fixed device array. */
int64_t lobpcg_gram_noalloc_max_bytes(void);

/* Basis update Y = beta * Y + alpha * S C (section 5.1, eqs. 10-11 and
 * Algorithm 8's basis update).  S: n x K (lds), C: K x N FP64 COLUMN-major (ldc >= K),
 * rounded to dtype inside the kernel; Y: n x N (ldy).  beta must be 0 or 1;
 * Y may not alias S. */
int lobpcg_update(int64_t n, int32_t K, int32_t N, int32_t dtype, const void* S, int64_t lds,
                  const double* C, int64_t ldc, double alpha, double beta, void* Y, int64_t ldy,
                  void* stream);

/* Bytes of workspace lobpcg_residual needs. */
int64_t lobpcg_residual_workspace(int64_t n, int32_t nx);

/* Residual and convergence test (Algorithm 8's residual and converged count, eq. 9):
 * R = AX - BX diag(theta) (BX may be NULL for B = I, meaning X);
 * W(:, nx-1-j) = dinv .* R(:, j) (reversed column order, section 5.1;
 * dinv NULL = identity; W may be NULL to skip);
 * rho_j = ||r_j||_2 / ((normA + |theta_j| normB) ||x_j||_2), sums in FP64.
 * theta, dinv, rho: device FP64 arrays (theta, rho length nx; dinv length n).
 * n_c_out (device int32, may be NULL): length of the leading run of
 * rho_j <= tol. */
int lobpcg_residual(int64_t n, int32_t nx, int32_t dtype, const void* AX, int64_t ldax,
                    const void* BX, int64_t ldbx, const void* X, int64_t ldx,
                    const double* theta, const double* dinv, void* W, int64_t ldw, double normA,
                    double normB, double tol, double* rho, int32_t* n_c_out, void* work,
                    void* stream);

/* Bytes of workspace lobpcg_spmm_residual needs. */
int64_t lobpcg_spmm_residual_workspace(int64_t n, int32_t nx);

/* The sparse product A X fused with Algorithm 8's residual and converged count for
 * B = I (eq. 9), the solver's path for recomputed A X: Y = A X formed row by row (CSR
 * A as in lobpcg_spmm; X: n x nx, ldx), stored to AX (ldax) only when AX != NULL;
 * R = Y - X diag(theta); W(:, nx-1-j) = dinv .* R(:, j) (reversed column order,
 * section 5.1; dinv NULL = identity; W must not be NULL nor alias X);
 * rho_j = ||r_j||_2 / ((normA + |theta_j|) ||x_j||_2) with FP64 sums; n_c_out as
 * lobpcg_residual.  The product's summation order is lobpcg_spmm's.  work:
 * lobpcg_spmm_residual_workspace(n, nx) bytes. */
int lobpcg_spmm_residual(int64_t n, const int64_t* rowptr, const int32_t* colind,
                         const void* values, int32_t dtype, const void* X, int64_t ldx,
                         int32_t nx, const double* theta, const double* dinv, void* W,
                         int64_t ldw, void* AX, int64_t ldax, double normA, double tol,
                         double* rho, int32_t* n_c_out, void* work, void* stream);

/* One RayleighRitzModified step (Algorithm 7) on the device, FP64.
 * GA, GB: n_s x n_s symmetric (column-major, ldg); GB is ignored when
 * use_ortho != 0 (S^T B S = I).  Reads n_x, n_c.  Outputs (device):
 *   C: n_s x (n_x + n_p) column-major (ldc >= n_s): [C_x, C_p];
 *   theta: n_s Ritz values ascending; theta_p: n_p x n_p column-major (ld n_x)
 *   block Q^T Theta_perp Q;
 * host outputs: *n_p, *flipped (1 when Cholesky was rejected: no coefficients
 * are produced), *cond (cond_1 of the scaled Cholesky factor; +inf when the
 * factorisation breaks down at a pivot that is not positive; 0 if unused).
 * tau_skip: section 5.3 threshold.
 * n_ident: 0, or the size of a leading block of GB that is exactly the identity
 * (the X and P blocks given by eqs. (12)-(14)); the Cholesky factor of Algorithm
 * 7 is then formed blockwise, factoring only the Schur complement of the
 * trailing n_s - n_ident block (the same factor in exact arithmetic).
 * Synchronises the stream. */
int lobpcg_rr_step(int32_t n_s, int32_t n_x, int32_t n_c, int32_t use_ortho,
                   int32_t lq_literal, int32_t n_ident, const double* GA, const double* GB,
                   int64_t ldg,
                   double tau_skip, double* C, int64_t ldc, double* theta, double* theta_p,
                   int32_t* n_p, int32_t* flipped, double* cond, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* LOBPCG_MI355X_STEPS_H */
