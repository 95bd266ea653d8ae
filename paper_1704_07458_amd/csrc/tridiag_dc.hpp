// Divide and conquer for the symmetric tridiagonal eigenproblem (tridiag_dc.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <cstdint>

namespace lobpcg {

int tridiag_dc_max_n();
int tridiag_dc_int_workspace();

// Eigen-decomposition T = Z diag(lam) Z^T of the n x n symmetric tridiagonal
// (d, e), n <= tridiag_dc_max_n(): lam ascending (may alias d, which is
// overwritten), Z column-major with leading dimension ldz.  Workspace (device):
// Qs, Dl, G, Y: n x n each with leading dimension ldz; vec4: 4 n doubles;
// iw: tridiag_dc_int_workspace() ints; rw: 2 tridiag_dc_max_n() doubles; rhoK: 64
// doubles.  fail: device int raised (never cleared) to 1 when a leaf's implicit
// QL iteration did not converge, to 2 when d or e held a non-finite value (each
// leaf block holding one is then solved as a zero block, and zeros are written
// over its e entries and any non-finite e at its boundaries, so that the merges
// read finite values only; the output is then not an eigendecomposition).  All
// on stream s; h runs the merge GEMMs.
void tridiag_dc(int n, double* d, const double* e, double* lam, double* Z, int64_t ldz,
                double* Qs, double* Dl, double* G, double* Y, double* vec4, int* iw, double* rw,
                double* rhoK, int* fail, rocblas_handle h, hipStream_t s);

}  // namespace lobpcg
