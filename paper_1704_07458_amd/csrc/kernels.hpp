// Launchers of the HIP kernels of the LOBPCG path (gfx950 / CDNA4).
// Every launcher takes device pointers and enqueues on `s`; none synchronises.
// Dense blocks are row-major with leading dimensions in elements unless a
// parameter says "cm" (column-major).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace lobpcg {

// Y = A X for CSR A (n x n) and X, Y (n x ncols).
template <typename T>
void launch_spmm(int64_t n, const int64_t* rowptr, const int32_t* colind, const T* vals,
                 const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, hipStream_t s);

// Gram G = L^T [R1 | R2] (L: n x m, R1: n x p1, R2: n x (p - p1)), FP64 output,
// column-major with leading dimension ldg: column j < p1 goes to column c1 + j of
// G1, the others to column c2 + j - p1 of G2.  Rows i < mirror_rows are also
// written transposed.  work must hold gram_workspace_bytes(n, m, p, fp32)
// bytes; gram_workspace_bound(n, m, p, fp32) covers every m' <= m, p' <= p.
int64_t gram_workspace_bytes(int64_t n, int m, int p, bool fp32);
int64_t gram_workspace_bound(int64_t n, int m, int p, bool fp32);
template <typename T>
void launch_gram(int64_t n, int m, int p, int p1, const T* L, int64_t ldl, const T* R1,
                 int64_t ldr1, const T* R2, int64_t ldr2, double* G1, int c1, double* G2, int c2,
                 int64_t ldg, int mirror_rows, void* work, hipStream_t s);

// The second stage of launch_gram on its own: G(i, c + j) = sum over the
// nparts partial tiles part[t][i * p + j] (row-major m x p each, summed in
// FP64 in a fixed order), columns j < p1 to G1 from c1, the rest to G2 from
// c2; mirror_rows as launch_gram.
template <typename P>
void launch_gram_reduce(int m, int p, int p1, int nparts, const P* part, double* G1, int c1,
                        double* G2, int c2, int64_t ldg, int mirror_rows, hipStream_t s);

// launch_gram with the split-K partial tiles in a fixed device array of
// kGramScratchBytes per GPU instead of a workspace (the split count is capped
// to fit); m * p * 8 > kGramScratchBytes is LOBPCG_ERR_ARG.  Calls that overlap
// on one GPU share that array and race.
constexpr int64_t kGramScratchBytes = int64_t(16) << 20;
template <typename T>
void launch_gram_noalloc(int64_t n, int m, int p, int p1, const T* L, int64_t ldl, const T* R1,
                         int64_t ldr1, const T* R2, int64_t ldr2, double* G1, int c1, double* G2,
                         int c2, int64_t ldg, int mirror_rows, hipStream_t s);
// Device address of that array on the current device (looked up once per device).
void* gram_scratch_address();

// Y = beta*Y + alpha * S C; C is FP64 column-major K x N (ldc).
template <typename T>
void launch_update(int64_t n, int K, int N, const T* S, int64_t lds, const double* C, int64_t ldc,
                   double alpha, double beta, T* Y, int64_t ldy, hipStream_t s);

// Residual R = AX - BX diag(theta); W(:, nx-1-j) = dinv .* R(:, j);
// rho_j per eq. (9); n_c[0] = leading run of rho_j <= tol, n_c[1] = 1 if any
// rho_j or theta_j is not finite.
int64_t residual_workspace_bytes(int64_t n, int nx);
template <typename T>
void launch_residual(int64_t n, int nx, const T* AX, int64_t ldax, const T* BX, int64_t ldbx,
                     const T* X, int64_t ldx, const double* theta, const double* dinv, T* W,
                     int64_t ldw, double normA, double normB, double tol, double* rho,
                     int32_t* n_c, void* work, hipStream_t s);

// out[j] = sum_i Y[i, j]^2 for j < ncols (FP64 accumulation, deterministic).
int64_t colsq_workspace_bytes(int64_t n, int ncols);
// A X fused with the residual for B = I: the sparse product over the n_x
// columns of X (row-major, ldx), then per row R = A X - X Theta written to W
// with reversed columns and the Jacobi factor dinv (may be NULL), A X to AX
// when AX != NULL, and criterion (9) with ||B|| = 1 as launch_residual.
// work: spmm_residual_workspace_bytes(n, nx) bytes.
int64_t spmm_residual_workspace_bytes(int64_t n, int nx);
template <typename T>
void launch_spmm_residual(int64_t n, const int64_t* rowptr, const int32_t* colind,
                          const T* vals, const T* X, int64_t ldx, int nx, const double* theta,
                          const double* dinv, T* W, int64_t ldw, T* AX, int64_t ldax,
                          double normA, double tol, double* rho, int32_t* n_c, void* work,
                          hipStream_t s);

template <typename T>
void launch_colsq(int64_t n, int ncols, const T* Y, int64_t ldy, double* out, void* work,
                  hipStream_t s);

// Jacobi preconditioner set-up: dinv[i] = 1 / (a_ii - sigma), sigma = 0 when every
// a_ii > 0, else the Gershgorin shift min_i(a_ii - sum_{j!=i}|a_ij|) - 1e-3 max_i sum_j |a_ij|.
void launch_jacobi_setup(int64_t n, const int64_t* rowptr, const int32_t* colind,
                         const double* vals, double* dinv, void* work, hipStream_t s);
int64_t jacobi_workspace_bytes(int64_t n);

// 2D strided copy / conversion of an n x ncols row-major block.
template <typename Tin, typename Tout>
void launch_copy2d(int64_t n, int ncols, const Tin* src, int64_t lds, Tout* dst, int64_t ldd,
                   hipStream_t s);

// Copy n x ncols row-major block with column reversal: dst(:, ncols-1-j) = src(:, j).
template <typename T>
void launch_copy2d_reverse(int64_t n, int ncols, const T* src, int64_t lds, T* dst, int64_t ldd,
                           hipStream_t s);

// Fill a row-major n x ncols block with Gaussian N(0,1) values: Philox-4x32-10
// (Salmon et al., SC'11) keyed by seed, counter (pair index, stream, 0), then
// Box-Muller on 53-bit uniforms.  Streams: 0 = the initial block drawn when
// none is given, 1 = the norm sketch of section 4.3.
constexpr uint32_t kStreamInitialBlock = 0;
constexpr uint32_t kStreamSketch = 1;
void launch_gaussian(int64_t n, int ncols, double* dst, int64_t ldd, uint64_t seed,
                     uint32_t stream, hipStream_t s);

// ---- small dense FP64 helpers (column-major, single workgroup or tiny grids) ----

// Implicit Gram blocks of eqs. (12)-(14): in the leading (nx+np) x (nx+np) block of
// GA set diag(theta) / 0 / theta_p (np x np, column-major, ld ldtp); in GB set I.
// GA and GB may each be null (that matrix is left untouched).
void launch_fill_implicit(int nx, int np, const double* theta, const double* theta_p,
                          int64_t ldtp, double* GA, double* GB, int64_t ldg, hipStream_t s);

// d_i = diag(G)_ii^-1/2 (0 when the diagonal entry is not positive); then
// Gout = D G D for the n x n block (in and out may alias).
void launch_diag_scale(int n, const double* G, int64_t ldg, double* d, double* Gout,
                       int64_t ldo, bool compute_d, hipStream_t s);

// cond_1 of upper-triangular R given R and Rinv (both column-major): writes
// ||R||_1 * ||Rinv||_1 to *cond.  scratch: 2n doubles.
void launch_cond1_upper(int n, const double* R, const double* Rinv, int64_t ld, double* cond,
                        double* scratch, hipStream_t s);

// Zero the strictly lower triangle of an n x n column-major matrix.
void launch_zero_lower(int n, double* A, int64_t ld, hipStream_t s);

// Row scaling: A(i, j) = d_i A(i, j) for an m x n column-major block.
void launch_row_scale(int m, int n, const double* d, double* A, int64_t lda, hipStream_t s);
// B = diag(d) A (m x n, column-major).
void launch_row_scale_copy(int m, int n, const double* d, const double* A, int64_t lda, double* B,
                           int64_t ldb, hipStream_t s);

// Column scaling: B(i, j) = A(i, j) * f(theta_j) for an m x n column-major block,
// mode 0: f = theta_j, mode 1: f = theta_j^-1/2.
void launch_col_scale(int m, int n, const double* A, int64_t lda, const double* theta, int mode,
                      double* B, int64_t ldb, hipStream_t s);

// Symmetrise: A = (A + A^T)/2 (n x n column-major).
void launch_symmetrize(int n, double* A, int64_t lda, hipStream_t s);

// Set A to the m x n identity-like pattern (1 on the diagonal).
void launch_set_identity(int m, int n, double* A, int64_t lda, hipStream_t s);
// y = -x (n values; y may be x).
void launch_negate(int n, const double* x, double* y, hipStream_t s);

// SVQB post-processing (Algorithms 4 and 6): theta ascending (n values).
// replace mode: theta_j <- max(theta_j, tau * max|theta|), keep all (keep = n).
// drop mode: keep only theta_j > tau * max|theta| (they are the trailing ones).
// Writes scale_j = theta_j^-1/2 for kept j (in the original index order), the
// index of the first kept column and the kept count to info[0], info[1].
void launch_svqb_theta(int n, double* theta, double tau, int drop, double* scale, int32_t* info,
                       hipStream_t s);

// Frobenius norm of (A - I) for an n x n column-major block, written to *out.
void launch_fro_minus_identity(int n, const double* A, int64_t lda, double* out, hipStream_t s);
// Frobenius norm of an m x n column-major block, written to *out.
void launch_fro(int m, int n, const double* A, int64_t lda, double* out, hipStream_t s);
// Householder tridiagonalisation of a symmetric n x n matrix (column-major,
// both triangles stored; n <= sytrd_max_n()) in one workgroup: d, e (n-1), tau
// (n-1) and the reflectors below the subdiagonal, in LAPACK's lower layout.
void launch_sytrd_lower(int n, double* A, int64_t lda, double* d, double* e, double* tau,
                        hipStream_t s);
int sytrd_max_n();
// Householder QR of the m x k block M (column-major, ld ldm, k <= m) and the
// explicit Q (m x k) in its place, in one workgroup (dgeqrf + dorgqr); valid
// when geqrf_orgqr_fits(m, k).
bool geqrf_orgqr_fits(int m, int k);
void launch_geqrf_orgqr(int m, int k, double* M, int64_t ldm, hipStream_t s);
// Z <- Q Z (n x n, column-major, ldz) with Q the product of the reflectors
// that launch_sytrd_lower left in A and tau (n <= sytrd_max_n()).
void launch_ormtr_lower(int n, const double* A, int64_t lda, const double* tau, double* Z,
                        int64_t ldz, hipStream_t s);
// out = sqrt(sum of v[0..n)) for a vector of squares.
void launch_sqrt_sum(int n, const double* v, double* out, hipStream_t s);

}  // namespace lobpcg
