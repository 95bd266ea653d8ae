/*
 * lobpcg.h -- C ABI of the MI355X (gfx950) robust LOBPCG library.
 *
 * Computes the k algebraically smallest eigenpairs of a symmetric-definite
 * pencil (A, B), A X = B X Lambda, A symmetric and B symmetric positive
 * definite (B = I when omitted), as defined in section 2 of Duersch, Shao,
 * Yang and Gu, "A Robust and Efficient Implementation of LOBPCG"
 * (arXiv 1704.07458): X minimises trace(X^T A X) subject to X^T B X = I
 * (eq. 1).  The iteration is the paper's Algorithm 8 (robust LOBPCG) with the
 * basis selection of Algorithms 5-7 and the backward-stable convergence test of
 * eq. (9); every step runs on the GPU in this library's HIP kernels (sparse
 * products, Gram blocks, basis updates, residuals) and in FP64 dense routines
 * on the device (Rayleigh-Ritz).
 *
 * Conventions shared by every entry point:
 *   - Dense blocks are ROW-MAJOR: element (i, j) of an n x m block with leading
 *     dimension ld lives at p[i * ld + j], ld >= m.  (Column-major only where
 *     stated.)
 *   - Sparse matrices are CSR with full symmetric storage, int64 row pointers
 *     (n + 1 entries, rowptr[0] = 0, rowptr[n] = nnz), int32 column indices
 *     sorted and unique within each row, FP64 values.
 *   - All work is enqueued on the HIP stream given in lobpcg_options.stream
 *     (NULL = the default stream); calls that return host data synchronise it.
 *   - Return value: 0 success, > 0 warning, < 0 error (codes below).  Nothing
 *     throws across this boundary.  lobpcg_last_error() gives a message for the
 *     last failing call on the calling thread.
 *   - A handle is not thread safe; distinct handles are independent.
 */
#ifndef LOBPCG_MI355X_H
#define LOBPCG_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define LOBPCG_OK 0
#define LOBPCG_NOT_CONVERGED 1  /* maxit reached; the n_converged leading pairs are valid */
#define LOBPCG_ERR_ARG (-1)     /* invalid argument or CSR structure */
#define LOBPCG_ERR_ALLOC (-2)   /* device allocation failed */
#define LOBPCG_ERR_HIP (-3)     /* a HIP runtime or ROCm library call failed */
#define LOBPCG_ERR_BREAKDOWN (-4) /* the search space collapsed (all of W and P dropped,
                                     or Cholesky of the initial block failed) */
#define LOBPCG_ERR_NONFINITE (-5) /* NaN or Inf appeared in a Ritz value or residual */
#define LOBPCG_ERR_CALLBACK (-6)  /* the preconditioner callback returned nonzero */
#define LOBPCG_ERR_STATE (-7)     /* call out of order (e.g. eigpairs before solve) */

/* Opaque solver handle; owns every device allocation it makes. */
typedef struct lobpcg_ctx* lobpcg_t;

/* Square sparse matrix in CSR form (see conventions).  on_device = 0: the three
 * arrays are host memory; 1: device memory.  lobpcg_create copies them. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* rowptr;
  const int32_t* colind;
  const double* values;
  int32_t on_device;
} lobpcg_csr;

/* Preconditioner callback: W = K^-1 R for the ncols columns of R (section 2:
 * W = K^-1 (A X - B X Theta) for any preconditioner K; Algorithm 8 applies it to
 * the unconverged residual columns).  R and W are DEVICE pointers to row-major
 * n x ncols blocks with leading dimensions ldr and ldw; dtype 0 = double,
 * 1 = float (FP32 phase of the precision-split mode).  The callback must enqueue
 * its work on `stream` (a hipStream_t) and return 0, or nonzero to abort the
 * solve with LOBPCG_ERR_CALLBACK.  W and R do not alias. */
typedef int (*lobpcg_precond_fn)(void* user, int64_t n, int32_t ncols, int32_t dtype,
                                 const void* R, int64_t ldr, void* W, int64_t ldw, void* stream);

/* Solver options.  Fill with lobpcg_default_options(), then override. */
typedef struct {
  int32_t block_size;        /* n_x >= k; 0 = k + ceil(k/10) (ten percent padding, section 6) */
  int32_t maxit;             /* iteration limit; 0 = 2000 (section 6) */
  int32_t precision;         /* 0 = FP64 throughout; 1 = precision split: FP32 sparse
                                products, Gram blocks and updates until the FP32 phase
                                converges at fp32_tol, then FP64 iterations to tol */
  int32_t precond;           /* 0 = none (K = I); 1 = Jacobi (diagonal of A, shifted to be
                                positive when it is not); 2 = the solve's callback */
  int32_t implicit_products; /* -1 (automatic) or 0: A X (and B X) are recomputed with the
                                sparse product after each update (on this GPU one SpMM costs
                                about half of an n x n_s by n_s x n_x product); 1: the implicit
                                updates A X = (A S) C_x, A P = (A S) C_p of section 5.2, which
                                keep A S = [A X, A P, A W] (two more n x n_s blocks of memory).
                                1 needs B = I (section 5.2: with B != I the updates are not
                                safe), else LOBPCG_ERR_ARG */
  int32_t lq_literal;        /* 0 = P built from the LQ of Z_1(:, n_c:n_x)^T Z_1perp; 1 = the first
                                n_x - n_c rows of the LQ of Z_1perp (Algorithm 7's P block) */
  double tau_ortho;          /* relative orthogonality tolerance of Algorithm 5; <= 0: 1e-12
                                (FP64), 1e-5 in the FP32 phase */
  double drop_factor;        /* tau_drop = drop_factor * n_u * eps (section 4.1); <= 0: 10 */
  double replace_factor;     /* tau_replace = replace_factor * n_u * eps (Algorithm 4); <= 0: 10 */
  double skip_factor;        /* tau_skip = skip_factor * eps; Cholesky of S^T B S is rejected when
                                cond_1(R)^3 * tau_skip > 1 (section 5.3); <= 0: 10 */
  double fp32_tol;           /* criterion (9) threshold ending the FP32 phase; <= 0: 1e-5 */
  uint64_t seed;             /* seed of the counter-based Gaussian generator (Philox-4x32-10,
                                Box-Muller): stream 0 gives the initial block when X0 is
                                NULL, stream 1 the sketch Omega of section 4.3 */
  void* stream;              /* hipStream_t for all work; NULL = default stream */
  /* Switches for the version ladder of section 6 (Figure 2); the defaults give
   * Algorithm 8. */
  int32_t ortho_mode;        /* 0 = orthoDrop (Algorithm 5, with basis truncation); 1 = ortho
                                (Algorithm 3, the Hetmaniuk-Lehoucq scheme: svqb on every inner
                                pass, no columns dropped) */
  int32_t force_ortho;       /* 1 = orthogonalise W from the first iteration and solve the
                                projected problem as a standard one (never the Cholesky path of
                                Algorithm 7), as the versions without skipped orthogonalisation */
  int32_t implicit_gram;     /* 1 = the X and P blocks of S^T A S and S^T B S from eqs. (12)-(14)
                                (default), except in a step that follows a Cholesky factor
                                with cond_1(R) > tau_skip^(-1/4) (see explicit_xp_steps);
                                0 = always computed explicitly (with A P and B P) */
  int32_t basic;             /* 1 = Algorithm 1, the basic LOBPCG, instead of Algorithm 8: W for
                                every column (no locking), every Gram block explicit,
                                Algorithm 2's Rayleigh-Ritz with no condition test and
                                P = S(:, n_x+1:end) C(n_x+1:end, 1:n_x); when S^T B S has no
                                Cholesky factor the solve stops with LOBPCG_ERR_BREAKDOWN (the
                                failure Algorithms 5-8 remove).  Other switches are ignored */
  int32_t largest;           /* 1 = the k largest eigenpairs instead (section 2: the Ritz values
                                ordered the other way round), computed as the k smallest of
                                (-A, B); lobpcg_eigpairs then returns descending values.  The
                                Jacobi preconditioner is built from -A (its diagonal shifted
                                positive).  lobpcg_adjoint rejects this mode (LOBPCG_ERR_ARG) */
  /* Device-memory hooks.  When both are non-NULL every device buffer the handle
   * owns (the matrices, the blocks, the projected-problem and rocBLAS /
   * rocSOLVER workspaces, the adjoint's temporaries) comes from
   * dev_alloc(bytes, alloc_user), which returns a device pointer aligned to at
   * least 256 bytes or NULL on failure (the call then fails with
   * LOBPCG_ERR_ALLOC), and is returned through dev_free(ptr, alloc_user) when
   * the handle no longer needs it (at the latest in lobpcg_destroy).  Memory is
   * used only on `stream` and, for Algorithm 7's P block, on one internal
   * stream that the handle synchronises before freeing.  Both NULL: hipMalloc /
   * hipFree.  Giving only one of them is LOBPCG_ERR_ARG. */
  void* (*dev_alloc)(size_t bytes, void* alloc_user);
  void (*dev_free)(void* ptr, void* alloc_user);
  void* alloc_user;
  /* Progress report of long solves: when non-NULL, called on the host after
   * every iteration (both phases of the precision split) with the iteration
   * count so far, the number of converged leading pairs and the phase (0 FP64,
   * 1 FP32).  It reads values the iteration copies to the host anyway: no
   * extra synchronisation.  It must not call into the handle. */
  void (*progress)(void* progress_user, int32_t iteration, int32_t n_converged, int32_t phase);
  void* progress_user;
} lobpcg_options;

/* Per-solve statistics. seconds_phase: 0 sparse products, 1 preconditioner,
 * 2 orthoDrop, 3 Gram blocks, 4 Rayleigh-Ritz, 5 basis update, 6 residual and
 * convergence test, 7 other (host-timed with stream synchronisation only when
 * profile_phases is set by lobpcg_set_profiling). */
typedef struct {
  int32_t iterations;         /* Algorithm 8 iterations (both phases in split mode) */
  int32_t n_converged;        /* leading pairs meeting criterion (9) at exit */
  int32_t ortho_switch_iter;  /* iteration at which useOrtho became true; -1 if never */
  int32_t fp32_iterations;    /* iterations of the FP32 phase (split mode) */
  int32_t fp64_iterations;    /* FP64 iterations */
  int32_t svqb_calls;         /* svqb + svqbDrop passes inside orthogonalisation */
  int32_t ortho_calls;        /* orthoDrop (or ortho, ortho_mode 1) calls */
  int32_t flips;              /* Cholesky rejections (0 or 1 per phase) */
  double norm_A_est;          /* ||A||_2 lower bound ||Omega A||_F / ||Omega||_F from the
                                 Gaussian sketch of section 4.3 (Omega: n_x x n, stream 1 of
                                 opt.seed; independent of X0, formed once per handle) */
  double norm_B_est;          /* same for B (1 when B = I) */
  double seconds_total;       /* wall time of lobpcg_solve */
  double seconds_phase[8];
  int32_t explicit_xp_steps;  /* steps whose X and P Gram blocks were computed explicitly instead
                                 of from eqs. (12)-(14) because the previous step's cond_1(R)
                                 exceeded tau_skip^(-1/4): [X P] is B-orthonormal only to about
                                 eps cond(R)^2 after such a step, and the implicit blocks would
                                 hide that error from the next step's Cholesky test */
  int32_t fp32_fallback;      /* precision split: 1 when the FP32 phase broke down (or met a
                                 non-finite value) and the FP64 phase took over from the last
                                 finite block (or from X0); 2 when it stopped because no further
                                 pair met fp32_tol within 200 iterations (FP32 residual floor) */
} lobpcg_info;

/* Fill *opt with the defaults documented above. */
void lobpcg_default_options(lobpcg_options* opt);

/* Create a solver for the k smallest eigenpairs of (A, B).
 * A: CSR, square, sorted unique columns (checked).  B: CSR of the same size or
 * NULL for B = I.  Symmetry is the caller's responsibility.  k >= 1 and
 * 3 * n_x <= n (the basis [X, P, W] must fit, section 4.2).  opt may be NULL.
 * Copies A and B to device memory owned by the handle.
 * Errors: LOBPCG_ERR_ARG, LOBPCG_ERR_ALLOC, LOBPCG_ERR_HIP. */
int lobpcg_create(lobpcg_t* out, const lobpcg_csr* A, const lobpcg_csr* B, int32_t k,
                  const lobpcg_options* opt);

/* Run Algorithm 8 to criterion (9) with threshold tol.
 * X0: row-major n x n_x initial block (ld = n_x), host memory when
 * x0_on_device = 0, device memory when 1; NULL = Gaussian N(0,1) block from
 * opt.seed (stream 0).  X0 is copied.
 * K: preconditioner callback (used when opt.precond = 2), K_user its argument.
 * info: may be NULL.
 * Returns LOBPCG_OK, LOBPCG_NOT_CONVERGED (maxit reached), or an error. */
int lobpcg_solve(lobpcg_t h, double tol, const double* X0, int32_t x0_on_device,
                 lobpcg_precond_fn K, void* K_user, lobpcg_info* info);

/* Copy out the leading `count` Ritz pairs (count <= n_x) of the last solve:
 * lambda (count values, ascending; descending with opt.largest), X (row-major n x count, leading dimension
 * ldx >= count, B-orthonormal columns) and rel_resid (criterion (9) per pair);
 * any output pointer may be NULL.  on_device = 0: host buffers; 1: device.
 * Errors: LOBPCG_ERR_STATE before a solve, LOBPCG_ERR_ARG. */
int lobpcg_eigpairs(lobpcg_t h, int32_t count, double* lambda, double* X, int64_t ldx,
                    double* rel_resid, int32_t on_device);

/* Gradient of a loss L(lambda_1..k, x_1..k) with respect to the stored values
 * of A (and of B) from the first `count` eigenpairs of the last solve (x_i
 * B-orthonormal).  First-order perturbation of A x = lambda B x:
 *   d lambda_i = x_i^T (dA - lambda_i dB) x_i,
 *   y_i = -sum_{j != i} x_j (x_j^T xbar_i) / (lambda_j - lambda_i),
 * split into the part inside the computed block and a projected conjugate-
 * gradient solve of Pi^T (A - lambda_i B) Pi z = -Pi^T xbar_i, y_i = Pi z, with
 * Pi = I - X X^T B (I - X X^T when B = I) for the rest.  For stored entry
 * p = (r, c), with the symmetric convention (a_rc and a_cr move together):
 *   grad[p]   = sum_i lambda_bar_i x_i(r) x_i(c) + 1/2 sum_i (y_i(r) x_i(c) + x_i(r) y_i(c)),
 *   grad_B[p] = sum_i a_i x_i(r) x_i(c) + 1/2 sum_i b_i (y_i(r) x_i(c) + x_i(r) y_i(c)),
 *   a_i = -(lambda_bar_i lambda_i + 1/2 xbar_i^T x_i), b_i = -lambda_i
 * (the xbar_i^T x_i term keeps x_i^T B x_i = 1).
 * lambda_bar: count values (host, may be NULL = 0); X_bar: row-major n x count
 * DEVICE block with leading dimension ld_xbar (may be NULL = 0); grad: nnz(A)
 * DEVICE values; grad_B: nnz(B) DEVICE values or NULL (must be NULL when B = I).
 * cg_tol: relative residual of the projected solve (<= 0: 1e-12); cg_maxit <= 0:
 * 10000.  cg_iters (host, may be NULL) receives the largest CG iteration count.
 * The CG residual is re-projected every step; a column whose curvature
 * p^T (projected operator) p is no longer positive has reached the rounding
 * floor and stops there.  Returns LOBPCG_OK, or LOBPCG_NOT_CONVERGED when
 * cg_maxit is reached with columns above cg_tol (the gradients are still
 * written, from the last iterate).  Errors: LOBPCG_ERR_STATE, LOBPCG_ERR_ARG. */
int lobpcg_adjoint(lobpcg_t h, int32_t count, const double* lambda_bar, const double* X_bar,
                   int64_t ld_xbar, double* grad, double* grad_B, double cg_tol,
                   int32_t cg_maxit, int32_t* cg_iters);

/* Complex Hermitian pencils (section 1: the method carries over to A = A^H,
 * B = B^H positive definite, with every transpose read as a conjugate
 * transpose).  CSR as lobpcg_csr, with the real and imaginary parts of the
 * stored values in two arrays of nnz doubles.  Symmetry (a_cr = conj(a_rc)) is
 * the caller's responsibility. */
typedef struct {
  int64_t n;
  int64_t nnz;
  const int64_t* rowptr;
  const int32_t* colind;
  const double* values_re;
  const double* values_im;
  int32_t on_device;
} lobpcg_zcsr;

/* Create a solver for the k smallest (opt.largest: largest) eigenpairs of the
 * complex Hermitian pencil (A, B), B = NULL for B = I.  The handle runs
 * Algorithm 8 on the real embedding Ahat = [Re A, -Im A; Im A, Re A] (order 2n,
 * 4 nnz(A) stored values; likewise Bhat) for 2k pairs with block width 2 n_x:
 * a complex eigenvalue is a double eigenvalue of the embedding, and the
 * stacked vectors of x and i x span its eigenspace.  The Jacobi preconditioner
 * is the embedding's (diag(Re A) twice); a preconditioner callback receives the
 * embedding's 2n-row real blocks.  lobpcg_kernel_stats, lobpcg_set_profiling
 * and lobpcg_dims (which reports n, k and n_x of the complex problem) accept
 * the handle; lobpcg_solve, lobpcg_eigpairs and lobpcg_adjoint reject it
 * (LOBPCG_ERR_ARG).  Requires 3 n_x <= n.  Errors as lobpcg_create. */
int lobpcg_create_hermitian(lobpcg_t* out, const lobpcg_zcsr* A, const lobpcg_zcsr* B, int32_t k,
                            const lobpcg_options* opt);

/* Run Algorithm 8 on the embedding from the paired block [X0, i X0].
 * X0_re, X0_im: row-major n x n_x real and imaginary parts of the complex
 * initial block (host memory when x0_on_device = 0, device when 1), both NULL
 * for the library's block: real parts from the first n rows and imaginary
 * parts from the last n rows of the seeded 2n x n_x Gaussian block (Philox
 * stream 0 of opt.seed).  The section 4.3 sketch is the embedding's (stream 1,
 * 2n x 2n_x), i.e. the complex Gaussian block with those halves.  info
 * reports the embedding's iteration (its n_converged counts real pairs).
 * Returns as lobpcg_solve. */
int lobpcg_solve_hermitian(lobpcg_t h, double tol, const double* X0_re, const double* X0_im,
                           int32_t x0_on_device, lobpcg_precond_fn K, void* K_user,
                           lobpcg_info* info);

/* The leading `count` (<= k) complex eigenpairs of the last solve: lambda
 * (ascending; descending with opt.largest), X_re / X_im (row-major n x count,
 * leading dimension ldx >= count, B-orthonormal columns: X^H B X = I) and
 * rel_resid (criterion (9) of each complex pair with the sketch norms).  The
 * pairs come from the 2k leading real Ritz vectors z_j = x(1:n) + i x(n+1:2n):
 * Q = the B-orthonormal basis of the k-dimensional range of Z^H B Z, then the
 * eigenpairs of Q^H A Q (complex Rayleigh-Ritz).  k must not split a cluster
 * of equal complex eigenvalues.  on_device = 0: host buffers; 1: device.
 * Errors: LOBPCG_ERR_STATE before a solve, LOBPCG_ERR_ARG. */
int lobpcg_eigpairs_hermitian(lobpcg_t h, int32_t count, double* lambda, double* X_re,
                              double* X_im, int64_t ldx, double* rel_resid, int32_t on_device);

/* Problem dimensions of a handle (any pointer may be NULL). */
int lobpcg_dims(lobpcg_t h, int64_t* n, int32_t* k, int32_t* n_x);

/* Free every device allocation of the handle.  NULL is ignored. */
void lobpcg_destroy(lobpcg_t h);

/* Message of the last failing call on this thread ("" if none). */
const char* lobpcg_last_error(void);

/* Per-kernel-class statistics of the solves run while collection is enabled,
 * for roofline accounting.  Each launch of a class is bracketed by HIP events
 * on the solver's stream; `work` sums the algorithmic work of the launches:
 *   kind 0 sparse products      work = bytes: nnz*(s_v+4) + 8*(n+1) + 2*n*ncols*s_v
 *   kind 1 Gram blocks          work = flops: 2*n*m*p
 *   kind 2 basis updates        work = flops: 2*n*K*N
 *   kind 3 residual + test      work = bytes: (3 or 4)*n*n_x*s_v + 8*n
 *   kind 4 Rayleigh-Ritz        work = 0 (dense FP64 on the projected pencil,
 *                               kinds 5-7 included)
 *   kind 5 tridiagonalisation   work = flops: (4/3) n_s^3 (one-workgroup Householder)
 *   kind 6 tridiagonal eigenproblem (divide and conquer)   work = 0
 *   kind 7 P-block QR and eigenvector back-transformation kernels  work = 0
 *   kind 8 Cholesky factor R of the scaled B-Gram matrix and R^-1 together
 *          (one workgroup, Algorithm 7)   work = flops: (2/3) n_s^3
 * (s_v = 8 for FP64, 4 for FP32 blocks.)  Kinds 5-8 are recorded only for
 * projected problems within the one-workgroup kernels' size range. */
#define LOBPCG_KERNEL_KINDS 9
typedef struct {
  int64_t launches;
  double seconds;
  double work;
} lobpcg_kernel_stat;

/* enable = 1: reset and start collecting; 0: stop.  out (may be NULL) receives
 * LOBPCG_KERNEL_KINDS entries indexed by kind, accumulated since the last reset. */
int lobpcg_kernel_stats(lobpcg_t h, int32_t enable, lobpcg_kernel_stat* out);

/* 1 = time the phases in lobpcg_info.seconds_phase (adds a stream
 * synchronisation per phase); 0 = off (default). */
int lobpcg_set_profiling(lobpcg_t h, int32_t on);

#ifdef __cplusplus
}
#endif

#endif /* LOBPCG_MI355X_H */
