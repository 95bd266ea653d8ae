// Cholesky factorisation G = R^T R and the inverse T = R^-1 in one workgroup
// (Algorithm 7: R from the scaled B-Gram matrix D S^T B S D, then R^-1 to form
// the standard eigenproblem R^-T (D S^T A S D) R^-1 and the coefficients).
//
// Right-looking Cholesky of the augmented block [G | I] by row operations:
// eliminating with the rows of R turns [G | I] into [R | R^-T], so the factor
// and the inverse come out of the same sweep (the flop count equals that of
// potrf plus trtri).  Panels are kCiNb rows.  In a panel every thread owns two
// columns of the panel rows (of G's trailing part or of the inverse's
// part left of the panel's end), held in registers; a step publishes the next
// pivot row through LDS, so a step costs one barrier.  After the panel the
// rows of R and of R^-T are final; the trailing matrix of G and the rows of
// R^-T below the panel receive the rank-kCiNb update from the panel rows
// staged in LDS.  R^-T is kept in the strict lower triangle of T while it is
// formed and written out transposed (R^-1, upper) as each panel completes.
// All sums run in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include <cmath>

#include "cholinv.hpp"
#include "common.hpp"

namespace lobpcg {
namespace {

constexpr int kCiThreads = 512;
constexpr int kCiNb = 32;
constexpr int kCiMaxN = 512;
// panel slots: G columns c0 .. n-1 at 0 .. n-c0-1, inverse columns 0 .. c0+w-1
// from the next multiple of 4 (aligned 16-byte reads in the trailing update)
constexpr int kCiSlots = kCiMaxN + kCiNb + 10;  // even; row stride 1092 words spreads LDS banks
constexpr int kCiPer = 2;  // slots 2t, 2t+1 per thread (two columns in registers)
static_assert(kCiSlots <= kCiPer * kCiThreads, "slots per thread");

__global__ __launch_bounds__(kCiThreads) void cholinv_upper_kernel(int n, double* __restrict__ A,
                                                                   int64_t lda,
                                                                   double* __restrict__ T,
                                                                   int64_t ldt,
                                                                   int32_t* __restrict__ info) {
  __shared__ __align__(16) double Pc[kCiNb * kCiSlots];  // Pc[i * kCiSlots + slot]: panel row i
  __shared__ double nxt[2 * kCiNb];        // the next pivot row, double-buffered
  const int t = threadIdx.x;
  // the strict lower triangle of R is zero; only G's upper triangle is read
  for (int c = 0; c < n - 1; ++c)
    for (int r = c + 1 + t; r < n; r += kCiThreads) A[r + (int64_t)c * lda] = 0.0;
  __syncthreads();  // the panel loads below also read (and ignore) these entries
  int failed_at = 0;
  for (int c0 = 0; c0 < n; c0 += kCiNb) {
    const int w = n - c0 < kCiNb ? n - c0 : kCiNb;
    const int na = n - c0;             // G columns c0 .. n-1
    const int eoff = (na + 3) & ~3;    // first inverse slot
    const int ne = c0 + w;             // inverse columns 0 .. c0+w-1
    // the panel rows into LDS with lanes running down each column's 32 rows
    // (coalesced): G columns c0 .. n-1, then the inverse's columns 0 .. c0-1
    // (its columns c0 .. c0+w-1 start as the identity and are not read)
    {
      const int cols = na + c0;
      for (int q = t; q < cols * kCiNb; q += kCiThreads) {
        const int i = q % kCiNb, k = q / kCiNb;
        const int ii = i < w ? i : w - 1;
        double v;
        int slot;
        if (k < na) {
          v = A[(c0 + ii) + (int64_t)(c0 + k) * lda];
          slot = k;
        } else {
          v = T[(c0 + ii) + (int64_t)(k - na) * ldt];
          slot = eoff + k - na;
        }
        Pc[i * kCiSlots + slot] = v;
      }
    }
    __syncthreads();
    bool isG[kCiPer], isE[kCiPer];
    int ce[kCiPer];  // inverse column of an inverse slot
    double p[kCiPer][kCiNb];
#pragma unroll
    for (int u = 0; u < kCiPer; ++u) {
      const int s = kCiPer * t + u;
      isG[u] = s < na;
      isE[u] = s >= eoff && s < eoff + ne;
      ce[u] = s - eoff;
      const bool fromT = isE[u] && ce[u] < c0;
      const int sl = (isG[u] || fromT) ? s : 0;
#pragma unroll
      for (int i = 0; i < kCiNb; ++i) {
        const double v = Pc[i * kCiSlots + sl];
        double x = 0.0;
        if (i < w) {
          if (isG[u])
            x = (s >= w || i <= s) ? v : 0.0;
          else if (fromT)
            x = v;
          else if (isE[u])
            x = (ce[u] - c0 == i) ? 1.0 : 0.0;
        }
        p[u][i] = x;
      }
    }
    if (t < kCiNb / kCiPer) {
      // slots s < w are the panel's diagonal-block columns
#pragma unroll
      for (int u = 0; u < kCiPer; ++u) {
        const int s = kCiPer * t + u;
        nxt[s] = (s < w) ? p[u][0] : 0.0;
        nxt[kCiNb + s] = 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kCiNb; ++j) {
      if (j < w && failed_at == 0) {
        const double* row = nxt + (j & 1) * kCiNb;
        const double piv = row[j];  // the same LDS word for every thread: a uniform branch
        if (!(piv > 0.0 && piv < INFINITY)) {
          failed_at = c0 + j + 1;
        } else {
          const double r = sqrt(piv);
          const double rinv = 1.0 / r;
          double pj[kCiPer];
#pragma unroll
          for (int u = 0; u < kCiPer; ++u) {
            pj[u] = (isG[u] && kCiPer * t + u == j) ? r : p[u][j] * rinv;
            p[u][j] = pj[u];
          }
#pragma unroll
          for (int i = j + 1; i < kCiNb; ++i) {
            const double rji = row[i] * rinv;
#pragma unroll
            for (int u = 0; u < kCiPer; ++u) p[u][i] = fma(-rji, pj[u], p[u][i]);
          }
#pragma unroll
          for (int u = 0; u < kCiPer; ++u) {
            const int s = kCiPer * t + u;
            if (isG[u] && s > j && s < w) nxt[((j + 1) & 1) * kCiNb + s] = p[u][j + 1];
          }
          __syncthreads();
        }
      }
    }
    if (failed_at != 0) break;
    // the panel rows of R and of R^-T are final: stage them in LDS (every
    // thread has finished reading the loaded panel at the last step's barrier)
#pragma unroll
    for (int u = 0; u < kCiPer; ++u) {
      const int s = kCiPer * t + u;
      if (isG[u] || isE[u]) {
#pragma unroll
        for (int i = 0; i < kCiNb; ++i) Pc[i * kCiSlots + s] = p[u][i];
      }
    }
    __syncthreads();
    // write-out (disjoint from the trailing update's rows >= c0 + w): rows of
    // R down each column; rows of R^-T transposed into R^-1, along its rows;
    // the staged R^-T entries of rows c0 .. c0+w-1 are cleared
    for (int q = t; q < na * kCiNb; q += kCiThreads) {
      const int i = q % kCiNb, k = q / kCiNb;
      if (i < w && (k >= w || i <= k)) A[(c0 + i) + (int64_t)(c0 + k) * lda] = Pc[i * kCiSlots + k];
    }
    for (int q = t; q < ne * kCiNb; q += kCiThreads) {
      const int c = q % ne, i = q / ne;
      if (i < w) T[c + (int64_t)(c0 + i) * ldt] = Pc[i * kCiSlots + eoff + c];
    }
    for (int q = t; q < c0 * kCiNb; q += kCiThreads) {
      const int i = q % kCiNb, c = q / kCiNb;
      if (i < w) T[(c0 + i) + (int64_t)c * ldt] = 0.0;
    }
    // trailing update: G22 -= R12^T R12 (upper triangle), E21 -= R12^T E1
    const int m = n - c0 - w;
    if (m > 0) {
      const int nbm = (m + 3) / 4, nbe = (ne + 3) / 4;
      const int ta = nbm * (nbm + 1) / 2;  // upper-triangle tiles of G22, column by column
      const int total = ta + nbm * nbe;
      for (int q = t; q < total; q += kCiThreads) {
        const bool tileG = q < ta;
        int bi, bj;
        if (tileG) {
          bj = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
          while (bj * (bj + 1) / 2 > q) --bj;
          while ((bj + 1) * (bj + 2) / 2 <= q) ++bj;
          bi = q - bj * (bj + 1) / 2;
        } else {
          bi = (q - ta) % nbm;
          bj = (q - ta) / nbm;
        }
        const int xs = w + 4 * bi;                     // slot of the tile's first row
        const int ys = tileG ? w + 4 * bj : eoff + 4 * bj;  // slot of its first column
        // the tile's current values from in-bounds (clamped) addresses, loaded
        // before the products so that their latency overlaps them
        const int r0 = c0 + w + 4 * bi;
        const int cb = tileG ? c0 + w + 4 * bj : 4 * bj;
        const int clim = tileG ? n : ne;
        double* base = tileG ? A : T;
        const int64_t ld = tileG ? lda : ldt;
        double old[4][4];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int c = min(cb + b, clim - 1);
#pragma unroll
          for (int a = 0; a < 4; ++a) old[a][b] = base[min(r0 + a, n - 1) + (int64_t)c * ld];
        }
        double acc[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
#pragma unroll 2
        for (int i = 0; i < w; ++i) {
          const double2* xr = reinterpret_cast<const double2*>(Pc + i * kCiSlots + xs);
          const double2* yr = reinterpret_cast<const double2*>(Pc + i * kCiSlots + ys);
          const double2 x01 = xr[0], x23 = xr[1], y01 = yr[0], y23 = yr[1];
          const double x[4] = {x01.x, x01.y, x23.x, x23.y};
          const double y[4] = {y01.x, y01.y, y23.x, y23.y};
#pragma unroll
          for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) acc[a][b] = fma(x[a], y[b], acc[a][b]);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int c = cb + b;
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            const int r = r0 + a;
            if (tileG) {
              if (c < n && r <= c) base[r + (int64_t)c * ld] = old[a][b] - acc[a][b];
            } else if (c < ne && r < n) {
              base[r + (int64_t)c * ld] = (c < c0 ? old[a][b] : 0.0) - acc[a][b];
            }
          }
        }
      }
      __syncthreads();
    }
  }
  if (t == 0) {
    info[0] = failed_at;
    info[1] = 0;
  }
}

}  // namespace

int cholinv_max_n() { return kCiMaxN; }

void launch_cholinv_upper(int n, double* A, int64_t lda, double* T, int64_t ldt, int32_t* info,
                          hipStream_t s) {
  LOBPCG_CHECK(n >= 1 && n <= kCiMaxN && lda >= n && ldt >= n, LOBPCG_ERR_ARG,
               "cholinv: sizes out of range");
  hipLaunchKernelGGL(cholinv_upper_kernel, dim3(1), dim3(kCiThreads), 0, s, n, A, lda, T, ldt, info);
  LOBPCG_HIP(hipGetLastError());
}

}  // namespace lobpcg
