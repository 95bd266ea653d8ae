// HIP kernels of the robust LOBPCG path for gfx950 (CDNA4, wave64).
//
//  spmm      CSR sparse x row-major block (HBM-bound): a wave owns 8 rows and
//            walks their nonzeros 64 at a time, lanes across columns,
//            XCD-contiguous row ranges.
//  gram      tall-skinny L^T R on MFMA (v_mfma_f64_16x16x4f64 / f32_16x16x4f32),
//            split-K over rows, deterministic FP64 second-stage sum.
//  update    row-tiled S C on MFMA (section 5.1 basis update).
//  residual  R = AX - BX Theta fused with the Jacobi preconditioner, the
//            reversed W store and FP64 column norms for criterion (9).
//  small     FP64 helpers for the projected (n_s x n_s) problem.
#include "wave.hpp"
#include "kernels.hpp"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"

namespace lobpcg {
namespace {

constexpr int kWave = 64;
constexpr int kXcds = 8;

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));
typedef int v4i __attribute__((ext_vector_type(4)));
// Config word of a raw buffer resource on gfx9-family chips (32-bit data,
// no swizzle): buffer loads take one per-lane offset and a scalar offset.
constexpr int kBufferConfig = 0x00020000;

// Workgroups are handed to the 8 XCDs round-robin.  Map the dispatch index so
// that each XCD works on one contiguous range of logical blocks: neighbouring
// rows then share that XCD's L2.  The map is a bijection on [0, nb).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int x = b % kXcds, i = b / kXcds;
  const int q = nb / kXcds, r = nb % kXcds;
  return x * q + (x < r ? x : r) + i;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// ------------------------------------------------------------------ SpMM
// Y = A X for CSR A and row-major X (ncols columns).  Grid: x = blocks of
// kSpmmRowsPerBlock rows (XCD-contiguous), y = column panels of 64*NC; each
// lane owns NC columns.  Each wave owns kSpmmRowsPerWave consecutive rows.  It
// loads their row pointers with one vector load, then the column indices and values
// of up to 64 nonzeros at a time (one per lane), and walks the nonzeros with
// each index and value broadcast from its lane (readlane, wave-uniform),
// issuing kSpmmBatch X-row loads before consuming them, so that a row costs a
// fraction of one memory latency instead of a chain of them.
constexpr int kSpmmRowsPerBlock = 32;
constexpr int kSpmmRowsPerWave = kSpmmRowsPerBlock / 4;
constexpr int kSpmmBatch = 8;

__device__ __forceinline__ int64_t readlane64(int64_t v, int l) {
  const uint64_t u = (uint64_t)v;
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), l);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double readlane_val(double v, int l) {
  return __builtin_bit_cast(double, readlane64(__builtin_bit_cast(int64_t, v), l));
}
__device__ __forceinline__ float readlane_val(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

template <typename T, int NC>
__global__ __launch_bounds__(256) void spmm_kernel(int64_t n,
                                                         const int64_t* __restrict__ rowptr,
                                                         const int32_t* __restrict__ colind,
                                                         const T* __restrict__ vals,
                                                         const T* __restrict__ X, int64_t ldx,
                                                         T* __restrict__ Y, int64_t ldy,
                                                         int ncols) {
  const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = uniform(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int col0 = blockIdx.y * (kWave * NC) + lane;
  const int64_t r0 = lb * kSpmmRowsPerBlock + (int64_t)wave * kSpmmRowsPerWave;
  if (r0 >= n) return;
  const int nr = (int)(n - r0 < kSpmmRowsPerWave ? n - r0 : kSpmmRowsPerWave);
  bool cok[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) cok[j] = col0 + kWave * j < ncols;
  const int64_t rpl = lane <= nr ? rowptr[r0 + lane] : 0;
  const int64_t pbeg = readlane64(rpl, 0), pend = readlane64(rpl, nr);
  int cr = 0;                       // current row (offset from r0), wave-uniform
  int64_t ce = readlane64(rpl, 1);  // end of the current row's nonzeros
  T acc[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) acc[j] = T(0);
  for (int64_t chunk = pbeg; chunk < pend; chunk += kWave) {
    const int cnt = (int)(pend - chunk < kWave ? pend - chunk : kWave);
    const int32_t cl = lane < cnt ? colind[chunk + lane] : 0;
    const T al = lane < cnt ? vals[chunk + lane] : T(0);
    for (int q = 0; q < cnt; q += kSpmmBatch) {
      T xb[kSpmmBatch][NC];
      T ab[kSpmmBatch];
#pragma unroll
      for (int u = 0; u < kSpmmBatch; ++u) {
        const bool ok = q + u < cnt;
        const int li = ok ? q + u : 0;
        const int64_t c = (int64_t)__builtin_amdgcn_readlane(cl, li);
        ab[u] = ok ? readlane_val(al, li) : T(0);
#pragma unroll
        for (int j = 0; j < NC; ++j)
          xb[u][j] = (ok && cok[j]) ? X[c * ldx + col0 + kWave * j] : T(0);
      }
#pragma unroll
      for (int u = 0; u < kSpmmBatch; ++u) {
        if (q + u < cnt) {
          const int64_t p = chunk + q + u;
          while (cr + 1 < nr && p >= ce) {  // the current row is complete (rows may be empty)
#pragma unroll
            for (int j = 0; j < NC; ++j) {
              if (cok[j]) Y[(r0 + cr) * ldy + col0 + kWave * j] = acc[j];
              acc[j] = T(0);
            }
            ++cr;
            ce = readlane64(rpl, cr + 1);
          }
#pragma unroll
          for (int j = 0; j < NC; ++j) acc[j] = fma(ab[u], xb[u][j], acc[j]);
        }
      }
    }
  }
  for (; cr < nr; ++cr) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (cok[j]) Y[(r0 + cr) * ldy + col0 + kWave * j] = acc[j];
      acc[j] = T(0);
    }
  }
}

// A X fused with the residual and the convergence sums (B = I): the sparse
// product of spmm_kernel over the n_x columns of X, and at the end of each row
// r, for each column j: res = (A X)(r, j) - theta_j X(r, j), W(r, n_x-1-j) =
// res * dinv[r] (res without dinv; the reversed W store of section 5.1),
// optionally AX(r, j), and the FP64 sums of res^2 and X(r, j)^2 over the
// workgroup's rows into part_r / part_x [n_x][block] (fixed order: each wave
// its rows in order, then the four waves in order).  X(r, :) is the row the
// diagonal entry gathered (loaded again for a row that stores no diagonal).
template <typename T, int NC>
__global__ __launch_bounds__(256) void spmm_residual_kernel(
    int64_t n, const int64_t* __restrict__ rowptr, const int32_t* __restrict__ colind,
    const T* __restrict__ vals, const T* __restrict__ X, int64_t ldx, int nx,
    const double* __restrict__ theta, const double* __restrict__ dinv, T* __restrict__ W,
    int64_t ldw, T* __restrict__ AX, int64_t ldax, double* __restrict__ part_r,
    double* __restrict__ part_x) {
  __shared__ double sr[4][kWave * NC], sx[4][kWave * NC];
  const int64_t lb = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = uniform(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int col0 = blockIdx.y * (kWave * NC) + lane;
  const int64_t r0 = lb * kSpmmRowsPerBlock + (int64_t)wave * kSpmmRowsPerWave;
  const int nr = r0 >= n ? 0 : (int)(n - r0 < kSpmmRowsPerWave ? n - r0 : kSpmmRowsPerWave);
  bool cok[NC];
  double th[NC], accr[NC], accx[NC];
  T acc[NC], xd[NC];
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    cok[j] = col0 + kWave * j < nx;
    th[j] = cok[j] ? theta[col0 + kWave * j] : 0.0;
    accr[j] = 0.0;
    accx[j] = 0.0;
    acc[j] = T(0);
    xd[j] = T(0);
  }
  bool diag = false;  // X(r, :) captured from the diagonal entry of the current row
  // row r0 + cr is complete: residual, stores and sums
  auto finish_row = [&](int cr) {
    const int64_t r = r0 + cr;
    const double dv = dinv ? dinv[r] : 1.0;
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (!cok[j]) continue;
      const int c = col0 + kWave * j;
      const double x = diag ? (double)xd[j] : (double)X[r * ldx + c];
      const double res = (double)acc[j] - x * th[j];
      accr[j] = fma(res, res, accr[j]);
      accx[j] = fma(x, x, accx[j]);
      W[r * ldw + (nx - 1 - c)] = (T)(res * dv);
      if (AX) AX[r * ldax + c] = acc[j];
    }
  };
  if (nr > 0) {
    const int64_t rpl = lane <= nr ? rowptr[r0 + lane] : 0;
    const int64_t pbeg = readlane64(rpl, 0), pend = readlane64(rpl, nr);
    int cr = 0;
    int64_t ce = readlane64(rpl, 1);
    for (int64_t chunk = pbeg; chunk < pend; chunk += kWave) {
      const int cnt = (int)(pend - chunk < kWave ? pend - chunk : kWave);
      const int32_t cl = lane < cnt ? colind[chunk + lane] : 0;
      const T al = lane < cnt ? vals[chunk + lane] : T(0);
      for (int q = 0; q < cnt; q += kSpmmBatch) {
        T xb[kSpmmBatch][NC];
        T ab[kSpmmBatch];
        int64_t cb[kSpmmBatch];
#pragma unroll
        for (int u = 0; u < kSpmmBatch; ++u) {
          const bool ok = q + u < cnt;
          const int li = ok ? q + u : 0;
          const int64_t c = (int64_t)__builtin_amdgcn_readlane(cl, li);
          cb[u] = c;
          ab[u] = ok ? readlane_val(al, li) : T(0);
#pragma unroll
          for (int j = 0; j < NC; ++j)
            xb[u][j] = (ok && cok[j]) ? X[c * ldx + col0 + kWave * j] : T(0);
        }
#pragma unroll
        for (int u = 0; u < kSpmmBatch; ++u) {
          if (q + u < cnt) {
            const int64_t p = chunk + q + u;
            while (cr + 1 < nr && p >= ce) {  // the current row is complete
              finish_row(cr);
#pragma unroll
              for (int j = 0; j < NC; ++j) acc[j] = T(0);
              diag = false;
              ++cr;
              ce = readlane64(rpl, cr + 1);
            }
            if (cb[u] == r0 + cr) {
#pragma unroll
              for (int j = 0; j < NC; ++j) xd[j] = xb[u][j];
              diag = true;
            }
#pragma unroll
            for (int j = 0; j < NC; ++j) acc[j] = fma(ab[u], xb[u][j], acc[j]);
          }
        }
      }
    }
    for (; cr < nr; ++cr) {
      finish_row(cr);
#pragma unroll
      for (int j = 0; j < NC; ++j) acc[j] = T(0);
      diag = false;
    }
  }
#pragma unroll
  for (int j = 0; j < NC; ++j) {
    sr[wave][lane + kWave * j] = accr[j];
    sx[wave][lane + kWave * j] = accx[j];
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int j = 0; j < NC; ++j) {
      if (!cok[j]) continue;
      const int t = lane + kWave * j;
      const double a = ((sr[0][t] + sr[1][t]) + sr[2][t]) + sr[3][t];
      const double b = ((sx[0][t] + sx[1][t]) + sx[2][t]) + sx[3][t];
      part_r[(int64_t)(col0 + kWave * j) * gridDim.x + lb] = a;
      part_x[(int64_t)(col0 + kWave * j) * gridDim.x + lb] = b;
    }
  }
}

// ------------------------------------------------------------------ MFMA
template <typename T>
struct Mfma;
// 16x16x4 MFMA lane layout (wave64), used by both kernels below:
//   A (16 x 4):  lane l holds A[l % 16][l / 16]
//   B (4 x 16):  lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l, accumulator element q holds D[row(l / 16, q)][l % 16] with
//                row = 4 * (l / 16) + q for f32 and row = l / 16 + 4 * q for f64
//                (the FP64 instruction interleaves the rows across lane groups).
template <>
struct Mfma<double> {
  using acc_t = v4d;
  __device__ static __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int lk, int q) { return lk + 4 * q; }
};
template <>
struct Mfma<float> {
  using acc_t = v4f;
  __device__ static __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static __forceinline__ int row(int lk, int q) { return 4 * lk + q; }
};

// ------------------------------------------------------------------ Gram
// Workgroup tile TM (m) x TP (p), TM, TP in {128, 64}: 2 x 2 waves, each wave a
// (TM/2) x (TP/2) register tile of MFMA 16x16x4 blocks; or one side 112 (seven
// blocks) with the four waves along the other side.  The row range is
// consumed in stages of kKB rows: each stage's L and R tiles are loaded with
// coalesced global loads into registers while the previous stage is
// multiplied out of LDS, then stored to the other LDS buffer (double
// buffering, one barrier per stage).  The tile size is chosen per launch to
// pad m and p least: the kernel is MFMA-bound, so padding is lost time.
// Grid: x = nsplit * tiles (tile index fastest, so workgroups that share a row
// range land together on one XCD).  Each workgroup sums its row range [k0, k1)
// and writes a partial tile to part[split][i][j].
constexpr int kGramTM = 128, kGramTP = 128, kKB = 16, kLdsPad = 2;

template <typename T, int TM, int TP, int WM, int WP = 4 / WM>
__global__ __launch_bounds__(kWave * WM * WP, 2) void gram_partial_kernel(
    int64_t n, int m, int p, int p1, const T* __restrict__ L, int64_t ldl,
    const T* __restrict__ R1, int64_t ldr1, const T* __restrict__ R2, int64_t ldr2,
    double* __restrict__ part, int tiles_m, int tiles_p, int64_t rows_per_split) {
  using acc_t = typename Mfma<T>::acc_t;
  // WM waves along m, WP along p (four waves, or seven 16-row stripes of a
  // 112 x 112 tile); each wave RM x CP of the tile in FA x FB MFMA blocks of 16 x 16
  constexpr int kThreads = kWave * WM * WP;
  constexpr int RM = TM / WM, CP = TP / WP;
  constexpr int FA = RM / 16, FB = CP / 16;
  static_assert(FA * 16 == RM && FB * 16 == CP, "16-row/column blocks");
  __shared__ T Ls[2][kKB][TM + kLdsPad];
  __shared__ T Rs[2][kKB][TP + kLdsPad];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int ntiles = tiles_m * tiles_p;
  const int split = lb / ntiles;
  const int tile = lb % ntiles;
  const int tm = tile / tiles_p, tp = tile % tiles_p;
  const int tid = threadIdx.x;
  const int wave = uniform(tid / kWave);
  const int lane = tid % kWave;
  const int wm = wave / WP, wp = wave % WP;
  const int li = lane & 15, lk = lane >> 4;

  const int64_t k0 = (int64_t)split * rows_per_split;
  const int64_t k1 = k0 + rows_per_split < n ? k0 + rows_per_split : n;

  // Global-load assignment: thread owns column ca of the L tile and rows
  // ra + RA i, and column cb of the R tile and rows rb + RB i.
  // (256 threads and a 112-wide tile leave threads 224.. idle)
  constexpr int RA = kThreads / TM, RB = kThreads / TP;
  constexpr int KA = kKB / RA, KBr = kKB / RB;  // rows per thread per stage
  const int ca = tid % TM, ra = tid / TM;
  const int cbt = tid % TP, rb = tid / TP;
  const int gca = tm * TM + ca;
  const bool okA = gca < m;
  const T* colA = L + (okA ? gca : 0);
  const int gcb = tp * TP + cbt;
  const bool okB = gcb < p;
  const T* colB;
  int64_t ldB;
  if (gcb < p1) {
    colB = R1 + gcb;
    ldB = ldr1;
  } else {
    colB = R2 + (okB ? gcb - p1 : 0);
    ldB = ldr2;
  }
  T ga[KA], gb[KBr];
  auto gload = [&](int64_t kb) {
#pragma unroll
    for (int i = 0; i < KA; ++i) {
      const int64_t row = kb + ra + RA * i;
      ga[i] = (ra < RA && row < k1 && okA) ? colA[row * ldl] : T(0);
    }
#pragma unroll
    for (int i = 0; i < KBr; ++i) {
      const int64_t row = kb + rb + RB * i;
      gb[i] = (rb < RB && row < k1 && okB) ? colB[row * ldB] : T(0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < KA; ++i)
      if (ra < RA) Ls[buf][ra + RA * i][ca] = ga[i];
#pragma unroll
    for (int i = 0; i < KBr; ++i)
      if (rb < RB) Rs[buf][rb + RB * i][cbt] = gb[i];
  };

  acc_t acc[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  const int64_t nst = (k1 - k0 + kKB - 1) / kKB;
  if (nst > 0) {
    gload(k0);
    sstore(0);
  }
  __syncthreads();
  for (int64_t st = 0; st < nst; ++st) {
    const int buf = (int)(st & 1);
    const bool more = st + 1 < nst;
    if (more) gload(k0 + (st + 1) * kKB);
#pragma unroll
    for (int s = 0; s < kKB / 4; ++s) {
      T a[FA], b[FB];
#pragma unroll
      for (int f = 0; f < FA; ++f) a[f] = Ls[buf][4 * s + lk][wm * RM + f * 16 + li];
#pragma unroll
      for (int f = 0; f < FB; ++f) b[f] = Rs[buf][4 * s + lk][wp * CP + f * 16 + li];
#pragma unroll
      for (int fa = 0; fa < FA; ++fa)
#pragma unroll
        for (int fb = 0; fb < FB; ++fb) acc[fa][fb] = Mfma<T>::mma(a[fa], b[fb], acc[fa][fb]);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
  }

  // Store the partial tile (FP64).
  double* out = part + (int64_t)split * m * p;
#pragma unroll
  for (int fa = 0; fa < FA; ++fa)
#pragma unroll
    for (int fb = 0; fb < FB; ++fb) {
      const int j = tp * TP + wp * CP + fb * 16 + li;
      if (j >= p) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = tm * TM + wm * RM + fa * 16 + Mfma<T>::row(lk, q);
        if (i < m) out[(int64_t)i * p + j] = (double)acc[fa][fb][q];
      }
    }
}

template <typename P>
__global__ __launch_bounds__(256) void gram_reduce_kernel(int m, int p, int p1, int nsplit,
                                                          const P* __restrict__ part,
                                                          double* __restrict__ G1, int c1,
                                                          double* __restrict__ G2, int c2,
                                                          int64_t ldg, int mirror_rows) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t mp = (int64_t)m * p;
  if (idx >= mp) return;
  const int i = (int)(idx / p), j = (int)(idx % p);
  // Four independent accumulators (more loads in flight), combined in a fixed order.
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int t = 0;
  for (; t + 4 <= nsplit; t += 4) {
    s0 += (double)part[(int64_t)t * mp + idx];
    s1 += (double)part[(int64_t)(t + 1) * mp + idx];
    s2 += (double)part[(int64_t)(t + 2) * mp + idx];
    s3 += (double)part[(int64_t)(t + 3) * mp + idx];
  }
  for (; t < nsplit; ++t) s0 += (double)part[(int64_t)t * mp + idx];
  const double s = (s0 + s1) + (s2 + s3);
  double* G = j < p1 ? G1 : G2;
  const int c = j < p1 ? c1 + j : c2 + (j - p1);
  G[i + (int64_t)c * ldg] = s;
  if (i < mirror_rows) G[c + (int64_t)i * ldg] = s;
}

struct GramPlan {
  int tm, tp;  // tile sizes (128, 112 or 64; at most one of them 112)
  int tiles_m, tiles_p, nsplit;
  int64_t rows_per_split;
};

// Two workgroups on each of 255 CUs: every workgroup of the split-K grid is
// resident at once even while a one-workgroup kernel holds a CU beside it.
constexpr int kGramTargetBlocks = 510;

// In FP32 the MFMA accumulators sum one split's rows in FP32; at most
// kGramFp32MaxRows rows per split (the splits' partial tiles are summed in
// FP64) keeps that rounding near sqrt(kGramFp32MaxRows) eps_32 (about 1e-5)
// even when the tiles alone would leave a single split of ~1e6 rows.
constexpr int64_t kGramFp32MaxRows = 8192;

GramPlan gram_plan(int64_t n, int m, int p, bool fp32) {
  GramPlan g;
  // the tile pair that pads m x p least (ties: the earlier, larger tiles); a
  // 112-wide side (seven 16-blocks, n_s = 330 -> 336, 2 n_w = 220 -> 224) takes
  // a 4 x 1 or 1 x 4 wave layout, so the other side must be 128 or 64
  auto padded = [](int x, int t) { return (int64_t)((x + t - 1) / t) * t; };
  static const int kPairs[9][2] = {{128, 128}, {128, 64}, {64, 128}, {64, 64}, {112, 112},
                                   {128, 112}, {112, 128}, {112, 64}, {64, 112}};
  int64_t best = -1;
  for (const auto& tt : kPairs) {
    const int64_t area = padded(m, tt[0]) * padded(p, tt[1]);
    if (best < 0 || area < best) {
      best = area;
      g.tm = tt[0];
      g.tp = tt[1];
    }
  }
  g.tiles_m = (m + g.tm - 1) / g.tm;
  g.tiles_p = (p + g.tp - 1) / g.tp;
  const int ntiles = g.tiles_m * g.tiles_p;
  // About kGramTargetBlocks workgroups (2 per CU) with at least 256 rows each.
  int64_t target = std::max<int64_t>(1, kGramTargetBlocks / std::max(ntiles, 1));
  int64_t max_by_rows = std::max<int64_t>(1, n / 256);
  int64_t ns = std::min(target, max_by_rows);
  if (fp32) ns = std::max(ns, (n + kGramFp32MaxRows - 1) / kGramFp32MaxRows);
  int64_t rps = (n + ns - 1) / ns;
  rps = round_up(std::max<int64_t>(rps, kKB), kKB);
  g.nsplit = (int)((n + rps - 1) / rps);
  if (g.nsplit < 1) g.nsplit = 1;
  g.rows_per_split = rps;
  return g;
}

// ------------------------------------------------------------------ update
// Y tile 128 rows x TN cols per workgroup, TN = 128, 112 or 64, whichever pads N
// least (N = n_x = 110 pads to 112): WR waves along the rows and 4 / WR along the
// columns (2 x 2 for 128 and 64, 4 x 1 with 32 x 112 per wave for 112), each a
// register tile of MFMA blocks.  K is
// consumed in stages of kKB: the S tile (128 rows x kKB, row segments of kKB
// contiguous elements) and the C tile (kKB x TN, column segments of C, which
// is column-major) go through double-buffered LDS as in the Gram kernel.
// Grid: x = row tiles * col tiles (col tile fastest).
constexpr int kUpdTM = 128, kUpdTN = 128, kUpdPad = 1;

template <typename T, int TN, int WR>
__global__ __launch_bounds__(256, 2) void update_kernel(int64_t n, int K, int N,
                                                     const T* __restrict__ S, int64_t lds,
                                                     const double* __restrict__ C, int64_t ldc,
                                                     T alpha, int beta1, T* __restrict__ Y,
                                                     int64_t ldy, int tiles_n) {
  using acc_t = typename Mfma<T>::acc_t;
  __shared__ T Ss[2][kUpdTM][kKB + kUpdPad];
  // WR waves along the rows, 4 / WR along the columns: each wave RW rows x CW
  // columns, FA x FB MFMA blocks
  constexpr int WC = 4 / WR, RW = kUpdTM / WR, CW = TN / WC;
  constexpr int FA = RW / 16, FB = CW / 16;
  static_assert(FA * 16 == RW && FB * 16 == CW, "16-row/column blocks");
  __shared__ T Cs[2][TN][kKB + kUpdPad];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t tr = lb / tiles_n;
  const int tc = lb % tiles_n;
  const int tid = threadIdx.x;
  const int wave = uniform(tid / kWave);
  const int lane = tid % kWave;
  const int wr = wave / WC, wc = wave % WC;
  const int li = lane & 15, lk = lane >> 4;

  // Global-load assignment: thread owns k offset kk of the stage and rows
  // (or columns) q0 + 16 i, i = 0..7.
  const int kk = tid % kKB;
  const int q0 = tid / kKB;
  constexpr int kPer = kUpdTM / 16, kPerC = TN / 16;
  const int rows_valid = (int)(n - tr * kUpdTM < kUpdTM ? n - tr * kUpdTM : kUpdTM);
  const int cols_valid = N - tc * TN < TN ? N - tc * TN : TN;
  const T* sbase = S + (tr * kUpdTM + q0) * lds + kk;
  const double* cbase = C + (int64_t)(tc * TN + q0) * ldc + kk;
  const int64_t sstep = 16 * lds, cstep = 16 * ldc;
  T gs[kPer], gc[kPerC];
  auto gload = [&](int kb) {
    const bool kok = kb + kk < K;
#pragma unroll
    for (int i = 0; i < kPer; ++i) {
      const int q = q0 + 16 * i;
      gs[i] = (kok && q < rows_valid) ? sbase[i * sstep + kb] : T(0);
    }
#pragma unroll
    for (int i = 0; i < kPerC; ++i) {
      const int q = q0 + 16 * i;
      gc[i] = (kok && q < cols_valid) ? (T)cbase[i * cstep + kb] : T(0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < kPer; ++i) Ss[buf][q0 + 16 * i][kk] = gs[i];
#pragma unroll
    for (int i = 0; i < kPerC; ++i) Cs[buf][q0 + 16 * i][kk] = gc[i];
  };

  acc_t acc[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};

  const int nst = (K + kKB - 1) / kKB;
  if (nst > 0) {
    gload(0);
    sstore(0);
  }
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    const bool more = st + 1 < nst;
    if (more) gload((st + 1) * kKB);
#pragma unroll
    for (int s = 0; s < kKB / 4; ++s) {
      T a[FA], b[FB];
#pragma unroll
      for (int f = 0; f < FA; ++f) a[f] = Ss[buf][wr * RW + f * 16 + li][4 * s + lk];
#pragma unroll
      for (int f = 0; f < FB; ++f) b[f] = Cs[buf][wc * CW + f * 16 + li][4 * s + lk];
#pragma unroll
      for (int fa = 0; fa < FA; ++fa)
#pragma unroll
        for (int fb = 0; fb < FB; ++fb) acc[fa][fb] = Mfma<T>::mma(a[fa], b[fb], acc[fa][fb]);
    }
    if (more) sstore(buf ^ 1);
    __syncthreads();
  }

#pragma unroll
  for (int fa = 0; fa < FA; ++fa)
#pragma unroll
    for (int fb = 0; fb < FB; ++fb) {
      const int j = tc * TN + wc * CW + fb * 16 + li;
      if (j >= N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = tr * kUpdTM + wr * RW + fa * 16 + Mfma<T>::row(lk, q);
        if (r < n) {
          T v = alpha * acc[fa][fb][q];
          if (beta1) v += Y[r * ldy + j];
          Y[r * ldy + j] = v;
        }
      }
    }
}

// The FP64 update with S fed by LDS DMA (global_load_lds_dwordx4): the S tile
// of a stage (128 rows x kKB) is 16 chunks of 8 rows, one 1 KB DMA each, and
// goes into one of three LDS buffers two stages ahead, with no staging
// registers and no LDS store instructions; C is loaded through registers one
// stage ahead as in update_kernel.  In a chunk, lane L holds row 8j + L/8 and
// the stage's k pair (L & 7) ^ (row & 7) (the XOR keeps the MFMA operand reads
// spread over the LDS banks); pairs past K read the last pair instead (C is
// zero there).  Needs K even and >= 2, lds even and S 16-byte aligned (the
// launcher checks).  Per iteration the C loads of stage st + 1 are issued
// before the DMA of stage st + 2, so the wait the compiler places for those C
// registers leaves only the newer DMA outstanding: stage st + 1's S, issued a
// stage earlier, has landed before the barrier.  Same products, same order
// of accumulation as update_kernel: the results are identical.
template <int TN, int WR>
__global__ __launch_bounds__(256, 2) void update_dma_kernel(int64_t n, int K, int N,
                                                            const double* __restrict__ S,
                                                            int64_t lds,
                                                            const double* __restrict__ C,
                                                            int64_t ldc, double alpha, int beta1,
                                                            double* __restrict__ Y, int64_t ldy,
                                                            int tiles_n) {
  using acc_t = v4d;
  typedef __attribute__((address_space(3))) void lds_void;
  __shared__ __align__(16) double Sd[3][kUpdTM * kKB];
  constexpr int WC = 4 / WR, RW = kUpdTM / WR, CW = TN / WC;
  constexpr int FA = RW / 16, FB = CW / 16;
  static_assert(FA * 16 == RW && FB * 16 == CW, "16-row/column blocks");
  static_assert(kKB == 16 && kUpdTM == 128, "8-row chunks of 16 doubles, four per wave");
  __shared__ double Cs[2][TN][kKB + kUpdPad];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t tr = lb / tiles_n;
  const int tc = lb % tiles_n;
  const int tid = threadIdx.x;
  const int wave = uniform(tid / kWave);
  const int lane = tid % kWave;
  const int wr = wave / WC, wc = wave % WC;
  const int li = lane & 15, lk = lane >> 4;
  const int rows_valid = (int)(n - tr * kUpdTM < kUpdTM ? n - tr * kUpdTM : kUpdTM);
  const int cols_valid = N - tc * TN < TN ? N - tc * TN : TN;
  auto dma_s = [&](int buf, int kb) {
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int j = wave + 4 * jj;
      const int row = 8 * j + (lane >> 3);
      const int p = (lane & 7) ^ (row & 7);
      const int r = row < rows_valid ? row : rows_valid - 1;
      const int k0 = kb + 2 * p + 1 < K ? kb + 2 * p : K - 2;
      __builtin_amdgcn_global_load_lds(S + (tr * kUpdTM + r) * lds + k0,
                                       (lds_void*)&Sd[buf][j * 8 * kKB], 16, 0, 0);
    }
  };
  const int kk = tid % kKB, q0 = tid / kKB;
  constexpr int kPerC = TN / 16;
  const double* cbase = C + (int64_t)(tc * TN + q0) * ldc + kk;
  const int64_t cstep = 16 * ldc;
  double gc[kPerC];
  auto gload_c = [&](int kb) {
    const bool kok = kb + kk < K;
#pragma unroll
    for (int i = 0; i < kPerC; ++i) {
      const int q = q0 + 16 * i;
      gc[i] = (kok && q < cols_valid) ? cbase[i * cstep + kb] : 0.0;
    }
  };
  auto sstore_c = [&](int buf) {
#pragma unroll
    for (int i = 0; i < kPerC; ++i) Cs[buf][q0 + 16 * i][kk] = gc[i];
  };
  acc_t acc[FA][FB];
#pragma unroll
  for (int a = 0; a < FA; ++a)
#pragma unroll
    for (int b = 0; b < FB; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
  const int nst = (K + kKB - 1) / kKB;
  dma_s(0, 0);
  gload_c(0);
  if (nst > 1) dma_s(1, kKB);
  sstore_c(0);
  __syncthreads();
  for (int st = 0; st < nst; ++st) {
    const bool more = st + 1 < nst;
    if (more) gload_c((st + 1) * kKB);
    if (st + 2 < nst) dma_s((st + 2) % 3, (st + 2) * kKB);
    const double* Sb = Sd[st % 3];
    const int cb = st & 1;
#pragma unroll
    for (int s4 = 0; s4 < kKB / 4; ++s4) {
      const int k = 4 * s4 + lk;
      double a[FA], b[FB];
#pragma unroll
      for (int f = 0; f < FA; ++f) {
        const int row = wr * RW + f * 16 + li;
        a[f] = Sb[row * kKB + 2 * ((k >> 1) ^ (row & 7)) + (k & 1)];
      }
#pragma unroll
      for (int f = 0; f < FB; ++f) b[f] = Cs[cb][wc * CW + f * 16 + li][k];
#pragma unroll
      for (int fa = 0; fa < FA; ++fa)
#pragma unroll
        for (int fb = 0; fb < FB; ++fb) acc[fa][fb] = Mfma<double>::mma(a[fa], b[fb], acc[fa][fb]);
    }
    if (more) sstore_c(cb ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int fa = 0; fa < FA; ++fa)
#pragma unroll
    for (int fb = 0; fb < FB; ++fb) {
      const int j = tc * TN + wc * CW + fb * 16 + li;
      if (j >= N) continue;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int64_t r = tr * kUpdTM + wr * RW + fa * 16 + Mfma<double>::row(lk, q);
        if (r < n) {
          double v = alpha * acc[fa][fb][q];
          if (beta1) v += Y[r * ldy + j];
          Y[r * ldy + j] = v;
        }
      }
    }
}

// ------------------------------------------------------------------ residual
// Grid: x = row blocks (kResRows rows each), y = column chunks of 64.
// Each thread owns one column; 4 waves stride over the block's rows.
constexpr int kResRows = 256;

template <typename T>
__global__ __launch_bounds__(256) void residual_kernel(
    int64_t n, int nx, const T* __restrict__ AX, int64_t ldax, const T* __restrict__ BX,
    int64_t ldbx, const T* __restrict__ X, int64_t ldx, const double* __restrict__ theta,
    const double* __restrict__ dinv, T* __restrict__ W, int64_t ldw, double* __restrict__ part_r,
    double* __restrict__ part_x) {
  __shared__ double sr[4][kWave], sx[4][kWave];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = uniform(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int j = blockIdx.y * kWave + lane;
  const bool ok = j < nx;
  const double th = ok ? theta[j] : 0.0;
  const int64_t r0 = (int64_t)lb * kResRows;
  const int64_t r1 = r0 + kResRows < n ? r0 + kResRows : n;
  double accr = 0.0, accx = 0.0;
  if (ok) {
    for (int64_t r = r0 + wave; r < r1; r += 4) {
      const double x = (double)X[r * ldx + j];
      const double bx = BX ? (double)BX[r * ldbx + j] : x;
      const double res = (double)AX[r * ldax + j] - bx * th;
      accr = fma(res, res, accr);
      accx = fma(x, x, accx);
      if (W) W[r * ldw + (nx - 1 - j)] = (T)(dinv ? res * dinv[r] : res);
    }
  }
  sr[wave][lane] = accr;
  sx[wave][lane] = accx;
  __syncthreads();
  if (wave == 0 && ok) {
    const double a = ((sr[0][lane] + sr[1][lane]) + sr[2][lane]) + sr[3][lane];
    const double b = ((sx[0][lane] + sx[1][lane]) + sx[2][lane]) + sx[3][lane];
    part_r[(int64_t)j * gridDim.x + lb] = a;
    part_x[(int64_t)j * gridDim.x + lb] = b;
  }
}

// Deterministic sums of column j's nblocks partials in one or two arrays
// (stored column after column: part[j * nblocks + block], so a column's
// partials are contiguous): one workgroup per column, each thread sums its
// fixed strided subset in order, then a fixed-order tree in LDS.  The loads
// go out in batches of kSumBatch per array before their adds (in the same
// order as one at a time, so the sums are the same bits): the partials of a
// 262144-row fused residual are 8192 per column, 32 per thread, and one round
// trip per add would make the kernel a chain of dependent loads.
constexpr int kSumBatch = 16;

template <int NA>
__device__ __forceinline__ void block_sum_columns(const double* const (&part)[NA], int nblocks,
                                                  int j, double* sbuf, double (&out)[NA]) {
  const int nt = blockDim.x;
  const double* col[NA];
  double a[NA];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    col[q] = part[q] + (int64_t)j * nblocks;
    a[q] = 0.0;
  }
  int t = threadIdx.x;
  for (; t + (kSumBatch - 1) * nt < nblocks; t += kSumBatch * nt) {
    double v[NA][kSumBatch];
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
      for (int u = 0; u < kSumBatch; ++u) v[q][u] = col[q][t + u * nt];
#pragma unroll
    for (int q = 0; q < NA; ++q)
#pragma unroll
      for (int u = 0; u < kSumBatch; ++u) a[q] += v[q][u];
  }
  for (; t < nblocks; t += nt)
#pragma unroll
    for (int q = 0; q < NA; ++q) a[q] += col[q][t];
#pragma unroll
  for (int q = 0; q < NA; ++q) {
    sbuf[threadIdx.x] = a[q];
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) sbuf[threadIdx.x] += sbuf[threadIdx.x + s];
      __syncthreads();
    }
    out[q] = sbuf[0];
    __syncthreads();
  }
}

// Grid: one workgroup per column.  rho_j of eq. (9).
__global__ __launch_bounds__(256) void residual_rho_kernel(
    int nx, int nblocks, const double* __restrict__ part_r, const double* __restrict__ part_x,
    const double* __restrict__ theta, double normA, double normB, double* __restrict__ rho) {
  (void)nx;
  __shared__ double sbuf[256];
  const int j = blockIdx.x;
  const double* const parts[2] = {part_r, part_x};
  double ab[2];
  block_sum_columns<2>(parts, nblocks, j, sbuf, ab);
  if (threadIdx.x == 0) rho[j] = sqrt(ab[0]) / ((normA + fabs(theta[j]) * normB) * sqrt(ab[1]));
}

// One workgroup: the leading run n_c[0] of rho_j <= tol and a non-finite flag n_c[1].
__global__ __launch_bounds__(256) void residual_nc_kernel(int nx, const double* __restrict__ rho,
                                                          const double* __restrict__ theta,
                                                          double tol, int32_t* __restrict__ n_c) {
  __shared__ int smin[256];
  __shared__ int sbad[256];
  int first_bad = nx, nonfinite = 0;
  for (int j = threadIdx.x; j < nx; j += blockDim.x) {
    const double r = rho[j];
    if (!(r <= tol) && j < first_bad) first_bad = j;
    if (!isfinite(r) || !isfinite(theta[j])) nonfinite = 1;
  }
  smin[threadIdx.x] = first_bad;
  sbad[threadIdx.x] = nonfinite;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      smin[threadIdx.x] = min(smin[threadIdx.x], smin[threadIdx.x + s]);
      sbad[threadIdx.x] = max(sbad[threadIdx.x], sbad[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && n_c) {
    n_c[0] = smin[0];
    n_c[1] = sbad[0];
  }
}

// ------------------------------------------------------------------ colsq
template <typename T>
__global__ __launch_bounds__(256) void colsq_kernel(int64_t n, int ncols, const T* __restrict__ Y,
                                                    int64_t ldy, double* __restrict__ part) {
  __shared__ double sq[4][kWave];
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int wave = uniform(threadIdx.x / kWave);
  const int lane = threadIdx.x % kWave;
  const int j = blockIdx.y * kWave + lane;
  const int64_t r0 = (int64_t)lb * kResRows;
  const int64_t r1 = r0 + kResRows < n ? r0 + kResRows : n;
  double acc = 0.0;
  if (j < ncols)
    for (int64_t r = r0 + wave; r < r1; r += 4) {
      const double y = (double)Y[r * ldy + j];
      acc = fma(y, y, acc);
    }
  sq[wave][lane] = acc;
  __syncthreads();
  if (wave == 0 && j < ncols)
    part[(int64_t)j * gridDim.x + lb] = ((sq[0][lane] + sq[1][lane]) + sq[2][lane]) + sq[3][lane];
}

// Grid: one workgroup per column.
__global__ __launch_bounds__(256) void colsq_finish_kernel(int ncols, int nblocks,
                                                           const double* __restrict__ part,
                                                           double* __restrict__ out) {
  (void)ncols;
  __shared__ double sbuf[256];
  const int j = blockIdx.x;
  const double* const parts[1] = {part};
  double a[1];
  block_sum_columns<1>(parts, nblocks, j, sbuf, a);
  if (threadIdx.x == 0) out[j] = a[0];
}

// ------------------------------------------------------------------ Jacobi
// Per row: diagonal, sum of |off-diagonal|, sum of all |a_ij|.
__global__ void jacobi_rows_kernel(int64_t n, const int64_t* __restrict__ rowptr,
                                   const int32_t* __restrict__ colind,
                                   const double* __restrict__ vals, double* __restrict__ diag,
                                   double* __restrict__ margin, double* __restrict__ absrow) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  double d = 0.0, off = 0.0, tot = 0.0;
  for (int64_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
    const double a = vals[p];
    tot += fabs(a);
    if (colind[p] == r) d += a;
    else off += fabs(a);
  }
  diag[r] = d;
  margin[r] = d - off;
  absrow[r] = tot;
}

// One workgroup: min of diag, min of margin, max of absrow.
__global__ __launch_bounds__(256) void jacobi_reduce_kernel(int64_t n, const double* diag,
                                                            const double* margin,
                                                            const double* absrow, double* out3) {
  __shared__ double s0[256], s1[256], s2[256];
  double mn = INFINITY, mg = INFINITY, mx = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += blockDim.x) {
    mn = fmin(mn, diag[r]);
    mg = fmin(mg, margin[r]);
    mx = fmax(mx, absrow[r]);
  }
  s0[threadIdx.x] = mn;
  s1[threadIdx.x] = mg;
  s2[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s0[threadIdx.x] = fmin(s0[threadIdx.x], s0[threadIdx.x + s]);
      s1[threadIdx.x] = fmin(s1[threadIdx.x], s1[threadIdx.x + s]);
      s2[threadIdx.x] = fmax(s2[threadIdx.x], s2[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out3[0] = s0[0];
    out3[1] = s1[0];
    out3[2] = s2[0];
  }
}

__global__ void jacobi_finish_kernel(int64_t n, const double* diag, const double* stats,
                                     double* dinv) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const double sigma = stats[0] > 0.0 ? 0.0 : stats[1] - 1e-3 * stats[2];
  dinv[r] = 1.0 / (diag[r] - sigma);
}

// ------------------------------------------------------------------ copies
template <typename Tin, typename Tout>
__global__ void copy2d_kernel(int64_t n, int ncols, const Tin* __restrict__ src, int64_t lds,
                              Tout* __restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int64_t r = idx / ncols;
  const int c = (int)(idx % ncols);
  dst[r * ldd + c] = (Tout)src[r * lds + c];
}

template <typename T>
__global__ void copy2d_reverse_kernel(int64_t n, int ncols, const T* __restrict__ src,
                                      int64_t lds, T* __restrict__ dst, int64_t ldd) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n * ncols) return;
  const int64_t r = idx / ncols;
  const int c = (int)(idx % ncols);
  dst[r * ldd + (ncols - 1 - c)] = src[r * lds + c];
}

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) counter-based generator.
__device__ __forceinline__ void philox_round(uint32_t c[4], const uint32_t k[2]) {
  const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
  const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
  const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
  const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
  const uint32_t n0 = hi1 ^ c[1] ^ k[0], n2 = hi0 ^ c[3] ^ k[1];
  c[0] = n0;
  c[1] = lo1;
  c[2] = n2;
  c[3] = lo0;
}

// Element pair (2q, 2q + 1) of the row-major block comes from the counter
// (q mod 2^32, q div 2^32, stream, 0) under the key (seed mod 2^32, seed div
// 2^32); stream 0 is the initial block, 1 the sketch of section 4.3.
__global__ void gaussian_kernel(int64_t n, int ncols, double* __restrict__ dst, int64_t ldd,
                                uint64_t seed, uint32_t stream) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = n * ncols;
  if (2 * idx >= total) return;
  uint32_t c[4] = {(uint32_t)idx, (uint32_t)(idx >> 32), stream, 0u};
  uint32_t k[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  for (int r = 0; r < 10; ++r) {
    philox_round(c, k);
    k[0] += 0x9E3779B9u;
    k[1] += 0xBB67AE85u;
  }
  // Two uniforms in (0, 1] from 64-bit words, then Box-Muller.
  const double u1 = ((double)(((uint64_t)c[0] << 32 | c[1]) >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(((uint64_t)c[2] << 32 | c[3]) >> 11) * 0x1.0p-53;
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 6.283185307179586 * u2;
  const int64_t e0 = 2 * idx, e1 = 2 * idx + 1;
  dst[(e0 / ncols) * ldd + e0 % ncols] = rad * cos(ang);
  if (e1 < total) dst[(e1 / ncols) * ldd + e1 % ncols] = rad * sin(ang);
}

// ------------------------------------------------------------------ small dense
__global__ void fill_implicit_kernel(int nx, int np, const double* __restrict__ theta,
                                     const double* __restrict__ theta_p, int64_t ldtp,
                                     double* __restrict__ GA, double* __restrict__ GB,
                                     int64_t ldg) {
  const int m = nx + np;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * m) return;
  const int i = (int)(idx % m), j = (int)(idx / m);
  double a = 0.0, b = (i == j) ? 1.0 : 0.0;
  if (i < nx && j < nx) a = (i == j) ? theta[i] : 0.0;
  else if (i >= nx && j >= nx) a = theta_p[(i - nx) + (int64_t)(j - nx) * ldtp];
  if (GA) GA[i + (int64_t)j * ldg] = a;
  if (GB) GB[i + (int64_t)j * ldg] = b;
}

__global__ void diag_d_kernel(int n, const double* __restrict__ G, int64_t ldg,
                              double* __restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double g = G[i + (int64_t)i * ldg];
  d[i] = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
}

__global__ void diag_scale_kernel(int n, const double* __restrict__ G, int64_t ldg,
                                  const double* __restrict__ d, double* __restrict__ Gout,
                                  int64_t ldo) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx % n), j = (int)(idx / n);
  Gout[i + (int64_t)j * ldo] = d[i] * G[i + (int64_t)j * ldg] * d[j];
}

// One wave per column: colsum[j] = sum_{i<=j} |A(i, j)| for A = R (slot 0) and Rinv (slot 1).
__global__ __launch_bounds__(256) void upper_colsum_kernel(int n, const double* __restrict__ R,
                                                           const double* __restrict__ Ri,
                                                           int64_t ld, double* __restrict__ out) {
  const int j = blockIdx.x * 4 + threadIdx.x / kWave;
  const int lane = threadIdx.x % kWave;
  if (j >= n) return;
  double a = 0.0, b = 0.0;
  for (int i = lane; i <= j; i += kWave) {
    a += fabs(R[i + (int64_t)j * ld]);
    b += fabs(Ri[i + (int64_t)j * ld]);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    a += __shfl_xor(a, off, kWave);
    b += __shfl_xor(b, off, kWave);
  }
  if (lane == 0) {
    out[j] = a;
    out[n + j] = b;
  }
}

// One workgroup: cond = max_j colsum_R(j) * max_j colsum_Rinv(j) (NaN propagates).
__global__ __launch_bounds__(256) void cond1_max_kernel(int n, const double* __restrict__ cs,
                                                        double* __restrict__ cond) {
  __shared__ double s0[256], s1[256];
  double m0 = 0.0, m1 = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    const double a = cs[j], b = cs[n + j];
    m0 = (a > m0 || a != a) ? a : m0;
    m1 = (b > m1 || b != b) ? b : m1;
  }
  s0[threadIdx.x] = m0;
  s1[threadIdx.x] = m1;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const double a = s0[threadIdx.x + s], b = s1[threadIdx.x + s];
      if (a > s0[threadIdx.x] || a != a) s0[threadIdx.x] = a;
      if (b > s1[threadIdx.x] || b != b) s1[threadIdx.x] = b;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) *cond = s0[0] * s1[0];
}

__global__ void zero_lower_kernel(int n, double* A, int64_t ld) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)n * n) return;
  const int i = (int)(idx % n), j = (int)(idx / n);
  if (i > j) A[i + (int64_t)j * ld] = 0.0;
}

__global__ void row_scale_kernel(int m, int n, const double* __restrict__ d, double* A,
                                 int64_t lda) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int i = (int)(idx % m), j = (int)(idx / m);
  A[i + (int64_t)j * lda] *= d[i];
}

__global__ void row_scale_copy_kernel(int m, int n, const double* __restrict__ d,
                                      const double* __restrict__ A, int64_t lda,
                                      double* __restrict__ B, int64_t ldb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int i = (int)(idx % m), j = (int)(idx / m);
  B[i + (int64_t)j * ldb] = d[i] * A[i + (int64_t)j * lda];
}

__global__ void col_scale_kernel(int m, int n, const double* __restrict__ A, int64_t lda,
                                 const double* __restrict__ theta, int mode,
                                 double* __restrict__ B, int64_t ldb) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int i = (int)(idx % m), j = (int)(idx / m);
  const double f = mode == 0 ? theta[j] : 1.0 / sqrt(theta[j]);
  B[i + (int64_t)j * ldb] = A[i + (int64_t)j * lda] * f;
}

// A <- (A + A^T) / 2 by pairs of 32 x 32 tiles (I, J), I <= J, one workgroup per
// pair: both tiles are read and written with lanes along columns (coalesced),
// the transposed tile through LDS.
constexpr int kSymTile = 32;
__global__ __launch_bounds__(256) void symmetrize_kernel(int n, double* A, int64_t lda) {
  __shared__ double tI[kSymTile][kSymTile + 1], tJ[kSymTile][kSymTile + 1];
  // pair index -> (I, J), J >= I, column by column of the upper tile triangle
  const int q = blockIdx.x;
  int J = (int)((sqrtf(8.0f * (float)q + 1.0f) - 1.0f) * 0.5f);
  while (J * (J + 1) / 2 > q) --J;
  while ((J + 1) * (J + 2) / 2 <= q) ++J;
  const int I = q - J * (J + 1) / 2;
  const int r = threadIdx.x % kSymTile, c0 = threadIdx.x / kSymTile;
  const int i0 = I * kSymTile, j0 = J * kSymTile;
  for (int c = c0; c < kSymTile; c += 256 / kSymTile) {
    // tI = A(i0 + r, j0 + c), tJ = A(j0 + r, i0 + c)
    tI[r][c] = (i0 + r < n && j0 + c < n) ? A[(i0 + r) + (int64_t)(j0 + c) * lda] : 0.0;
    tJ[r][c] = (j0 + r < n && i0 + c < n) ? A[(j0 + r) + (int64_t)(i0 + c) * lda] : 0.0;
  }
  __syncthreads();
  for (int c = c0; c < kSymTile; c += 256 / kSymTile) {
    // A(i0 + r, j0 + c) and its mirror A(j0 + c, i0 + r) both become the mean
    if (i0 + r < n && j0 + c < n) A[(i0 + r) + (int64_t)(j0 + c) * lda] = 0.5 * (tI[r][c] + tJ[c][r]);
    if (j0 + r < n && i0 + c < n) A[(j0 + r) + (int64_t)(i0 + c) * lda] = 0.5 * (tJ[r][c] + tI[c][r]);
  }
}

__global__ void set_identity_kernel(int m, int n, double* A, int64_t lda) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (int64_t)m * n) return;
  const int i = (int)(idx % m), j = (int)(idx / m);
  A[i + (int64_t)j * lda] = (i == j) ? 1.0 : 0.0;
}

__global__ void negate_kernel(int n, const double* __restrict__ x, double* __restrict__ y) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = -x[i];
}

// theta ascending.  The eigenvalues above the threshold form a trailing run.
__global__ __launch_bounds__(256) void svqb_theta_kernel(int n, double* theta, double tau, int drop,
                                                         double* scale, int32_t* info) {
  __shared__ double smax[256];
  double mx = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) mx = fmax(mx, fabs(theta[j]));
  smax[threadIdx.x] = mx;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
    __syncthreads();
  }
  const double thr = tau * smax[0];
  __syncthreads();
  __shared__ int sfirst[256];
  int first = n;
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double t = theta[j];
    if (drop) {
      if (t > thr) {
        first = min(first, j);
        scale[j] = 1.0 / sqrt(t);
      } else {
        scale[j] = 0.0;
      }
    } else {
      if (t < thr) t = thr;
      theta[j] = t;
      scale[j] = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
      first = 0;
    }
  }
  sfirst[threadIdx.x] = first;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sfirst[threadIdx.x] = min(sfirst[threadIdx.x], sfirst[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    const int f = drop ? sfirst[0] : 0;
    info[0] = f;
    info[1] = n - f;
  }
}

__global__ __launch_bounds__(256) void fro_kernel(int m, int n, const double* __restrict__ A,
                                                  int64_t lda, int minus_identity, double* out) {
  __shared__ double s[256];
  double acc = 0.0;
  const int64_t total = (int64_t)m * n;
  for (int64_t idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int i = (int)(idx % m), j = (int)(idx / m);
    double v = A[i + (int64_t)j * lda];
    if (minus_identity && i == j) v -= 1.0;
    acc = fma(v, v, acc);
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(s[0]);
}

__global__ __launch_bounds__(256) void sqrt_sum_kernel(int n, const double* __restrict__ v,
                                                       double* out) {
  __shared__ double s[256];
  double acc = 0.0;
  for (int j = threadIdx.x; j < n; j += blockDim.x) acc += v[j];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int st = blockDim.x / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st) s[threadIdx.x] += s[threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sqrt(s[0]);
}

// ------------------------------------------------------------------ tridiagonal
// Householder reduction of a symmetric n x n matrix (column-major, both
// triangles stored) to tridiagonal form, in one workgroup and one launch:
// A = Q T Q^T with Q = H(0) H(1) ... H(n-2), H(i) = I - tau_i v_i v_i^T,
// v_i(i+1) = 1, v_i(i+2:n) stored in A(i+2:n, i), d = diag(T), e = subdiag(T).
// All sums run in a fixed order (deterministic).
//
// Blocked Householder tridiagonalisation (lower), one workgroup, after the
// panel scheme of LAPACK's dsytrd / dlatrd: within a panel of kTrdNb columns
// the trailing matrix is left as it was at the panel start, each step
// corrects its column and its product A v with the panel's reflectors and
// their w vectors (V, W, kept in LDS), and the trailing matrix receives the
// rank-2 kTrdNb update V W^T + W V^T once per panel.  A step therefore reads
// the trailing matrix once (the product) instead of reading and writing it.
// Output as LAPACK's dsytrd with uplo = 'L': d, e, tau, reflectors below the
// subdiagonal of A.
constexpr int kTrdThreads = 1024;
constexpr int kTrdMaxN = 512;
constexpr int kTrdNb = 16;
static_assert(kTrdMaxN <= kTrdThreads, "one row per thread in the column steps");

__device__ __forceinline__ double wave_sum(double v) { return wave64_sum(v); }

// Workgroup sum with one barrier: wave sums into red[wave], then every thread
// adds the partials in the same fixed order.  Callers alternate between two
// red buffers with a barrier between successive uses of the same one.
__device__ __forceinline__ double trd_block_sum(double v, double* red) {
  v = wave_sum(v);
  if (threadIdx.x % kWave == 0) red[threadIdx.x / kWave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kTrdThreads / kWave; ++q) s += red[q];
  return s;
}

template <bool kPairs>
__global__ __launch_bounds__(kTrdThreads) void sytrd_lower_kernel(int n, double* __restrict__ A,
                                                                  int64_t lda,
                                                                  double* __restrict__ d,
                                                                  double* __restrict__ e,
                                                                  double* __restrict__ tau) {
  __shared__ double V[kTrdNb * kTrdMaxN];  // V[k * kTrdMaxN + r]: reflector k of the panel
  __shared__ double W[kTrdNb * kTrdMaxN];  // W[k * kTrdMaxN + r]
  __shared__ double cv[kTrdMaxN];          // the current column, updated
  __shared__ double pp[2 * kTrdThreads];   // partial products per column group
  __shared__ double yv[2 * kTrdNb];        // W^T v, V^T v
  __shared__ double redA[kTrdThreads / kWave], redB[kTrdThreads / kWave];
  __shared__ double pdet[3][kTrdNb];       // the panel's d, e (beta), tau, stored at its end
  const int t = threadIdx.x;
  const int lane = t % kWave, wave = t / kWave;
  constexpr int nwaves = kTrdThreads / kWave;
  // n <= kTrdMaxN <= kTrdThreads: thread t owns row i + t of column i in (a),
  // and keeps A(i + 1 + t, i + 1) from step i's product for step i + 1.
  double pre = 0.0;
  bool have_pre = false;
  for (int i0 = 0; i0 < n - 1; i0 += kTrdNb) {
    const int nbp = n - 1 - i0 < kTrdNb ? n - 1 - i0 : kTrdNb;
    for (int j = 0; j < nbp; ++j) {
      const int i = i0 + j;
      double* col = A + (int64_t)i * lda;
      const double* vj = V + j * kTrdMaxN;
      // (a) column i with the panel's deferred update; |A(i+2:n, i)|^2
      double part = 0.0;
      {
        const int r = i + t;
        if (r < n) {
          double a = have_pre ? pre : col[r];
          // unrolled so that the LDS loads of several reflectors are in flight
#pragma unroll 4
          for (int k = 0; k < j; ++k)
            a -= V[k * kTrdMaxN + r] * W[k * kTrdMaxN + i] + W[k * kTrdMaxN + r] * V[k * kTrdMaxN + i];
          cv[r] = a;
          if (r >= i + 2) part = fma(a, a, part);
        }
      }
      const double xnorm2 = trd_block_sum(part, redA);
      // (b) the reflector H = I - tau v v^T with H A(i+1:n, i) = beta e_1
      const double alpha = cv[i + 1];
      double taui = 0.0, beta = alpha, scal = 0.0;
      if (xnorm2 > 0.0) {
        beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
        taui = (beta - alpha) / beta;
        scal = 1.0 / (alpha - beta);
      }
      // n <= kTrdThreads: thread t owns row i0 + t of the reflector.  The
      // reflector and d, e, tau reach global memory only at the panel's end (a
      // barrier waits for outstanding stores; there they overlap the update).
      const int rv = i0 + t;
      double vst = 0.0;
      if (rv < n) {
        if (rv == i + 1) {
          vst = 1.0;
        } else if (rv >= i + 2) {
          vst = cv[rv] * scal;
        }
        V[j * kTrdMaxN + rv] = vst;
      }
      if (t == 0) {
        pdet[0][j] = cv[i];
        pdet[1][j] = beta;
        pdet[2][j] = taui;
      }
      __syncthreads();
      // (c) y1 = W^T v, y2 = V^T v over the panel's earlier columns (one wave
      // per value) and the partial products of the unupdated trailing matrix.
      for (int q = wave; q < 2 * j; q += nwaves) {
        const double* M = q < j ? W + q * kTrdMaxN : V + (q - j) * kTrdMaxN;
        double acc = 0.0;
        int r = i + 1 + lane;
        // four rows' reads in flight at a time, summed in row order
        for (; r + 3 * kWave < n; r += 4 * kWave) {
          double mv[4], vv[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            mv[u] = M[r + u * kWave];
            vv[u] = vj[r + u * kWave];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc = fma(mv[u], vv[u], acc);
        }
        for (; r < n; r += kWave) acc = fma(M[r], vj[r], acc);
        acc = wave_sum(acc);
        if (lane == 0) yv[q] = acc;
      }
      // Rows are taken in pairs [rb + 2q, rb + 2q + 1] (rb = i + 1, rounded down
      // to even when kPairs) so that one 16-byte load covers two rows: the
      // product is bound by load instructions, not bytes.  Column groups split
      // the columns; a thread sums its rows over its group's columns.
      constexpr int kR = kPairs ? 2 : 1;
      const int rb = kPairs ? ((i + 1) & ~1) : i + 1;
      const int nq = (n - rb + kR - 1) / kR;
      const int q_pass = ((nq + kWave - 1) / kWave) * kWave;
      const int groups = kTrdThreads / q_pass;  // 2..16 column groups
      const int rows_pass = kR * q_pass;
      {
        const int g = uniform(t / q_pass), qq = t % q_pass;  // q_pass: whole waves
        // column i + 1 is not modified again within the panel: keep its raw
        // entry for the next step (thread t owns row i + 1 + t there)
        have_pre = j + 1 < nbp && i + 1 + t < n;
        if (have_pre) pre = A[(int64_t)(i + 1) * lda + i + 1 + t];
        if (g < groups) {
          const int r0 = rb + kR * qq;
          double acc0 = 0.0, acc1 = 0.0;
          if (r0 < n) {
            // batches of 8 independent loads, issued before their sums
            const int64_t step = (int64_t)groups * lda;
            const double* ap = A + (int64_t)(i + 1 + g) * lda + r0;
            int c = i + 1 + g;
            // An odd last row takes the pair path too: its partner row n lies in
            // the column's padding (lda even, so lda > n), and that partner's sum
            // goes to a slot that is never read.
            if (kPairs) {
              // buffer loads: the lane's byte offset in one register, the
              // batch's column offsets scalar (the launcher keeps lda n 8 < 2^31)
              const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
                  A, (short)0, (int)(lda * n * (int64_t)sizeof(double)), kBufferConfig);
              int voff = (int)(((int64_t)c * lda + r0) * (int64_t)sizeof(double));
              const int cstep = (int)(step * (int64_t)sizeof(double));
              for (; c + 7 * groups < n; c += 8 * groups) {
                // the batch's v entries first, all in flight together with the
                // matrix loads (one LDS latency per batch, not one per column)
                double vc[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) vc[u] = vj[c + u * groups];
                v4i raw[8];
#pragma unroll
                for (int u = 0; u < 8; ++u)
                  raw[u] = __builtin_amdgcn_raw_buffer_load_b128(rs, voff, u * cstep, 0);
                voff += 8 * cstep;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                  const v2d av = __builtin_bit_cast(v2d, raw[u]);
                  acc0 = fma(av.x, vc[u], acc0);
                  acc1 = fma(av.y, vc[u], acc1);
                }
              }
              ap = A + (int64_t)c * lda + r0;
              for (; c < n; c += groups) {
                const double2 av = *reinterpret_cast<const double2*>(ap);
                acc0 = fma(av.x, vj[c], acc0);
                acc1 = fma(av.y, vj[c], acc1);
                ap += step;
              }
            } else {
              for (; c + 7 * groups < n; c += 8 * groups) {
                double av[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) av[u] = ap[u * step];
                ap += 8 * step;
#pragma unroll
                for (int u = 0; u < 8; ++u) acc0 = fma(av[u], vj[c + u * groups], acc0);
              }
              for (; c < n; c += groups) {
                acc0 = fma(*ap, vj[c], acc0);
                ap += step;
              }
            }
          }
          pp[g * rows_pass + kR * qq] = acc0;
          if (kPairs) pp[g * rows_pass + kR * qq + 1] = acc1;
        }
      }
      __syncthreads();
      // (d) p = tau (A v - V y1 - W y2);  w = p - (tau/2)(p^T v) v
      double dp = 0.0;
      for (int r = i + 1 + t; r < n; r += kTrdThreads) {
        const int rr = r - rb;
        double pr = 0.0;
#pragma unroll 4
        for (int q = 0; q < groups; ++q) pr += pp[q * rows_pass + rr];
#pragma unroll 4
        for (int k = 0; k < j; ++k)
          pr -= V[k * kTrdMaxN + r] * yv[k] + W[k * kTrdMaxN + r] * yv[j + k];
        pr *= taui;
        W[j * kTrdMaxN + r] = pr;
        dp = fma(pr, vj[r], dp);
      }
      const double pv = trd_block_sum(dp, redB);
      const double alpha2 = -0.5 * taui * pv;
      for (int r = i0 + t; r < n; r += kTrdThreads)
        W[j * kTrdMaxN + r] = r >= i + 1 ? fma(alpha2, vj[r], W[j * kTrdMaxN + r]) : 0.0;
      __syncthreads();
    }
    // (e) A(c0:n, c0:n) -= V W^T + W V^T = -[V W] [W V]^T on MFMA
    // (v_mfma_f64_16x16x4f64, K = 2 nbp in 4-deep slices): one wave per 16 x 16
    // tile of the lower triangle; an off-diagonal tile is stored at both of its
    // symmetric positions, so the matrix stays exactly symmetric there.
    {
      // the panel's reflectors (v below the subdiagonal, beta on it) and d, e, tau
      if (t < nbp) {
        d[i0 + t] = pdet[0][t];
        e[i0 + t] = pdet[1][t];
        tau[i0 + t] = pdet[2][t];
      }
      for (int k = 0; k < nbp; ++k) {
        const int r = i0 + t;  // rows i0 + k + 1 .. n - 1 of column i0 + k
        if (r >= i0 + k + 1 && r < n)
          A[(int64_t)(i0 + k) * lda + r] = r == i0 + k + 1 ? pdet[1][k] : V[k * kTrdMaxN + r];
      }
      const int c0 = i0 + nbp;
      const int ntl = (n - c0 + 15) / 16;
      const int kk = 2 * nbp;
      const int li = lane % 16, lq = lane / 16;
      for (int tix = wave; tix < ntl * (ntl + 1) / 2; tix += nwaves) {
        // tile (tr, tc), tr >= tc, from its index in the packed lower triangle
        int tr = (int)((sqrtf(8.0f * (float)tix + 1.0f) - 1.0f) * 0.5f);
        while ((tr + 1) * (tr + 2) / 2 <= tix) ++tr;
        while (tr * (tr + 1) / 2 > tix) --tr;
        const int tc = tix - tr * (tr + 1) / 2;
        const int R0 = c0 + 16 * tr, C0 = c0 + 16 * tc;
        // accumulator layout: element q of lane l is (R0 + l/16 + 4q, C0 + l%16)
        const int cd = C0 + li;
        v4d acc;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rd = R0 + lq + 4 * q;
          acc[q] = (rd < n && cd < n) ? A[(int64_t)cd * lda + rd] : 0.0;
        }
        // operands: A(row R0 + l%16, k = 4s + l/16), B(k = 4s + l/16, column C0 + l%16),
        // four slices' operands loaded before their MFMAs (a masked slice adds 0 x 0)
        const int ra = R0 + li;
        for (int s0 = 0; s0 < (kk + 3) / 4; s0 += 4) {  // wave-uniform trip count
          double a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = 4 * (s0 + u) + lq;
            a[u] = 0.0;
            b[u] = 0.0;
            if (k < kk) {
              if (ra < n) a[u] = -(k < nbp ? V[k * kTrdMaxN + ra] : W[(k - nbp) * kTrdMaxN + ra]);
              if (cd < n) b[u] = k < nbp ? W[k * kTrdMaxN + cd] : V[(k - nbp) * kTrdMaxN + cd];
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u], b[u], acc, 0, 0, 0);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int rd = R0 + lq + 4 * q;
          if (rd < n && cd < n) {
            A[(int64_t)cd * lda + rd] = acc[q];
            if (tr != tc) A[(int64_t)rd * lda + cd] = acc[q];
          }
        }
      }
    }
    __syncthreads();
  }
  if (t == 0) d[n - 1] = A[(int64_t)(n - 1) * lda + (n - 1)];
}

// Z <- Q Z with Q = H(0) H(1) ... H(n-2) from sytrd_lower_kernel (the
// back-transformation of the tridiagonal eigenvectors, LAPACK's dormtr with
// side = 'L', uplo = 'L', trans = 'N').  A workgroup owns kOrmCols columns of
// Z; 32 lanes of one wave own a column and hold its rows l, l + 32, ... in
// registers, so applying a reflector is a shuffle reduction and an update in
// registers, with no workgroup barrier.  Reflectors are staged through LDS
// kOrmBatch at a time (last one first), each batch loaded into registers
// while the previous one is applied.  Staged v_j is zero above row j + 1 and
// beyond n, so the per-reflector loops need no bounds.
constexpr int kOrmCols = 8;
constexpr int kOrmBatch = 16;
constexpr int kOrmThreads = 32 * kOrmCols;
constexpr int kOrmRows = kTrdMaxN / 32;                  // rows per lane
constexpr int kOrmLoad = kTrdMaxN / kOrmThreads;         // staged rows per thread per reflector

__global__ __launch_bounds__(kOrmThreads) void ormtr_lower_kernel(int n, const double* __restrict__ A,
                                                                  int64_t lda,
                                                                  const double* __restrict__ tau,
                                                                  double* __restrict__ Z,
                                                                  int64_t ldz) {
  __shared__ double Vb[kOrmBatch * kTrdMaxN];
  __shared__ double tb[kOrmBatch];
  const int t = threadIdx.x;
  const int cc = t / 32, l32 = t % 32;
  const int c = blockIdx.x * kOrmCols + cc;
  double z[kOrmRows];
#pragma unroll
  for (int q = 0; q < kOrmRows; ++q) {
    const int r = l32 + 32 * q;
    z[q] = (c < n && r < n) ? Z[(int64_t)c * ldz + r] : 0.0;
  }
  // staged value of reflector j at row r
  auto vload = [&](int j, int r) -> double {
    if (j < 0 || r >= n || r <= j) return 0.0;
    return r == j + 1 ? 1.0 : A[(int64_t)j * lda + r];
  };
  double nb[kOrmBatch][kOrmLoad];
  double ntau = 0.0;
  {
    const int hi = n - 2;
#pragma unroll
    for (int b = 0; b < kOrmBatch; ++b)
#pragma unroll
      for (int q = 0; q < kOrmLoad; ++q) nb[b][q] = vload(hi - b, t + kOrmThreads * q);
    if (t < kOrmBatch && hi - t >= 0) ntau = tau[hi - t];
  }
  for (int hi = n - 2; hi >= 0; hi -= kOrmBatch) {
    __syncthreads();  // the previous batch is no longer read
#pragma unroll
    for (int b = 0; b < kOrmBatch; ++b)
#pragma unroll
      for (int q = 0; q < kOrmLoad; ++q) Vb[b * kTrdMaxN + t + kOrmThreads * q] = nb[b][q];
    if (t < kOrmBatch) tb[t] = hi - t >= 0 ? ntau : 0.0;
    __syncthreads();
    const int hn = hi - kOrmBatch;
    if (hn >= 0) {
#pragma unroll
      for (int b = 0; b < kOrmBatch; ++b)
#pragma unroll
        for (int q = 0; q < kOrmLoad; ++q) nb[b][q] = vload(hn - b, t + kOrmThreads * q);
      ntau = (t < kOrmBatch && hn - t >= 0) ? tau[hn - t] : 0.0;
    }
    const int nbat = hi + 1 < kOrmBatch ? hi + 1 : kOrmBatch;
    for (int b = 0; b < nbat; ++b) {
      const double* v = Vb + b * kTrdMaxN + l32;
      double sdot = 0.0;
#pragma unroll
      for (int q = 0; q < kOrmRows; ++q) sdot = fma(v[32 * q], z[q], sdot);
      sdot = half32_sum(sdot);
      const double f = tb[b] * sdot;
#pragma unroll
      for (int q = 0; q < kOrmRows; ++q) z[q] = fma(-f, v[32 * q], z[q]);
    }
  }
  if (c < n) {
#pragma unroll
    for (int q = 0; q < kOrmRows; ++q) {
      const int r = l32 + 32 * q;
      if (r < n) Z[(int64_t)c * ldz + r] = z[q];
    }
  }
}

// ------------------------------------------------------------------ QR
// Householder QR of an m x k block (column-major, ld) followed by the
// explicit Q (m x k): LAPACK's dgeqrf + dorgqr conventions (beta = -sign(alpha)
// |x|, tau = (beta - alpha) / beta, v = x / (alpha - beta), H = I when the
// column below the diagonal is zero).  One workgroup, the block in registers:
// thread (c, g) holds column c, rows [g kQrRows, (g + 1) kQrRows).  A step is a
// norm from kQrGroups partials, the reflector broadcast through LDS, one dot
// product per column reduced over the kQrGroups row groups through LDS, and a register
// update.  Q overwrites the block.  m <= kQrMaxM, k <= kQrCols.
constexpr int kQrThreads = 1024;
constexpr int kQrCols = 128;
constexpr int kQrGroups = kQrThreads / kQrCols;
constexpr int kQrRows = 32;
constexpr int kQrMaxM = kQrGroups * kQrRows;

__global__ __launch_bounds__(kQrThreads) void geqrf_orgqr_kernel(int m, int k,
                                                                 double* __restrict__ M,
                                                                 int64_t ldm) {
  constexpr int kWaves = kQrThreads / kWave;
  __shared__ double colb[2][kQrMaxM];           // column j of the step, double-buffered
  __shared__ double vw[kWaves][kQrRows];        // per wave: the reflector on its rows
  __shared__ double fw[kWaves][kQrRows];        // per wave: column j's final entries
  __shared__ double vbuf[3][kQrMaxM];           // reflectors while Q is formed
  __shared__ double wpart[2][kQrGroups][kQrCols];
  __shared__ double taus[kQrCols];
  const int t = threadIdx.x;
  const int lane = t % kWave, wave = t / kWave;
  const int c = t % kQrCols, g = t / kQrCols;  // a wave lies in one row group
  const int r0 = g * kQrRows;
  double a[kQrRows];
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) {
    const int r = r0 + q;
    a[q] = (c < k && r < m) ? M[(int64_t)c * ldm + r] : 0.0;
  }
  for (int r = t; r < kQrMaxM; r += kQrThreads) colb[0][r] = colb[1][r] = 0.0;
  __syncthreads();
  if (c == 0) {
#pragma unroll
    for (int q = 0; q < kQrRows; ++q) colb[0][r0 + q] = a[q];
  }
  __syncthreads();
  // ---- factorisation, two barriers per column: every wave forms the
  // reflector of column j from the staged column (identical values in all
  // waves) and writes it for its own rows to its LDS slice, where lane q
  // handles row r0 + q (so the masks are per lane); the slice is read back by
  // the same wave only, after a wave-level fence.
  for (int j = 0; j < k; ++j) {
    const double* col = colb[j & 1];
    double sq = 0.0;
    for (int r = j + 1 + lane; r < m; r += kWave) sq = fma(col[r], col[r], sq);
    sq = wave_sum(sq);
    const double alpha = col[j];
    double tj = 0.0, beta = alpha, scal = 0.0;
    if (sq > 0.0) {
      beta = -copysign(sqrt(alpha * alpha + sq), alpha);
      tj = (beta - alpha) / beta;
      scal = 1.0 / (alpha - beta);
    }
    if (t == 0) taus[j] = tj;
    if (lane < kQrRows) {
      const int r = r0 + lane;
      const double x = col[r];
      const double v = r > j ? x * scal : (r == j ? 1.0 : 0.0);
      vw[wave][lane] = v;
      fw[wave][lane] = r > j ? v : (r == j ? beta : x);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const double* vq = vw[wave];
    if (c == j) {
#pragma unroll
      for (int q = 0; q < kQrRows; ++q) a[q] = fw[wave][q];
    }
    const bool act = c > j && c < k;
    if (act) {
      double sdot = 0.0;
#pragma unroll
      for (int q = 0; q < kQrRows; ++q) sdot = fma(vq[q], a[q], sdot);
      wpart[j & 1][g][c] = sdot;
    }
    __syncthreads();
    if (act) {
      double w = 0.0;
#pragma unroll
      for (int q = 0; q < kQrGroups; ++q) w += wpart[j & 1][q][c];
      const double f = tj * w;
#pragma unroll
      for (int q = 0; q < kQrRows; ++q) a[q] = fma(-f, vq[q], a[q]);
      if (c == j + 1) {
#pragma unroll
        for (int q = 0; q < kQrRows; ++q) colb[(j + 1) & 1][r0 + q] = a[q];
      }
    }
    __syncthreads();
  }
  // reflectors (below the diagonal) back to M; Q is built from them below
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) {
    const int r = r0 + q;
    if (c < k && r < m) M[(int64_t)c * ldm + r] = a[q];
  }
  __syncthreads();
  // ---- Q = H(0) ... H(k-1) I(:, 0:k), last reflector first, one barrier per
  // reflector: reflector j - 1 is staged (third buffer) while j is applied,
  // the partial sums alternate between two buffers
  auto vval = [&](int j, int r) -> double {
    if (j < 0 || r < j || r >= m) return 0.0;
    return r == j ? 1.0 : M[(int64_t)j * ldm + r];
  };
  if (t < kQrMaxM) vbuf[(k - 1) % 3][t] = vval(k - 1, t);
  double pre = t < kQrMaxM ? vval(k - 2, t) : 0.0;
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) a[q] = (c < k && r0 + q == c) ? 1.0 : 0.0;
  __syncthreads();
  for (int j = k - 1; j >= 0; --j) {
    const double* vb = vbuf[j % 3];
    if (c < k) {
      double sdot = 0.0;
#pragma unroll
      for (int q = 0; q < kQrRows; ++q) sdot = fma(vb[r0 + q], a[q], sdot);
      wpart[j & 1][g][c] = sdot;
    }
    if (j >= 1 && t < kQrMaxM) {
      vbuf[(j - 1) % 3][t] = pre;
      pre = vval(j - 2, t);
    }
    __syncthreads();
    if (c < k) {
      double w = 0.0;
#pragma unroll
      for (int q = 0; q < kQrGroups; ++q) w += wpart[j & 1][q][c];
      const double f = taus[j] * w;
#pragma unroll
      for (int q = 0; q < kQrRows; ++q) a[q] = fma(-f, vb[r0 + q], a[q]);
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < kQrRows; ++q) {
    const int r = r0 + q;
    if (c < k && r < m) M[(int64_t)c * ldm + r] = a[q];
  }
}

inline unsigned blocks_for(int64_t total, int threads = 256) {
  return (unsigned)((total + threads - 1) / threads);
}

}  // namespace

// ====================================================================== launchers
template <typename T>
void launch_spmm(int64_t n, const int64_t* rowptr, const int32_t* colind, const T* vals,
                 const T* X, int64_t ldx, T* Y, int64_t ldy, int ncols, hipStream_t s) {
  if (n == 0 || ncols == 0) return;
  const unsigned gx = (unsigned)((n + kSpmmRowsPerBlock - 1) / kSpmmRowsPerBlock);
  if (ncols <= 64) {
    hipLaunchKernelGGL((spmm_kernel<T, 1>), dim3(gx, 1), dim3(256), 0, s, n, rowptr, colind, vals,
                       X, ldx, Y, ldy, ncols);
  } else if (ncols <= 128) {
    hipLaunchKernelGGL((spmm_kernel<T, 2>), dim3(gx, 1), dim3(256), 0, s, n, rowptr, colind, vals,
                       X, ldx, Y, ldy, ncols);
  } else {
    const unsigned gy = (unsigned)((ncols + 255) / 256);
    hipLaunchKernelGGL((spmm_kernel<T, 4>), dim3(gx, gy), dim3(256), 0, s, n, rowptr, colind,
                       vals, X, ldx, Y, ldy, ncols);
  }
  LOBPCG_HIP(hipGetLastError());
}

int64_t gram_workspace_bytes(int64_t n, int m, int p, bool fp32) {
  if (n == 0 || m == 0 || p == 0) return 0;
  const GramPlan g = gram_plan(n, m, p, fp32);
  return (int64_t)g.nsplit * m * p * (int64_t)sizeof(double);
}

namespace {
template <typename T>
void launch_gram_plan(const GramPlan& g, int64_t n, int m, int p, int p1, const T* L, int64_t ldl,
                      const T* R1, int64_t ldr1, const T* R2, int64_t ldr2, double* G1, int c1,
                      double* G2, int c2, int64_t ldg, int mirror_rows, void* work,
                      hipStream_t s) {
  const int nsplit = n > 0 ? g.nsplit : 0;
  double* part = static_cast<double*>(work);
  if (nsplit > 0) {
    const unsigned grid = (unsigned)(nsplit * g.tiles_m * g.tiles_p);
    const T* R2e = R2 ? R2 : R1;
    const int64_t ldr2e = R2 ? ldr2 : ldr1;
#define LOBPCG_GRAM_LAUNCH(TMv, TPv, WMv)                                                    \
  hipLaunchKernelGGL((gram_partial_kernel<T, TMv, TPv, WMv>), dim3(grid), dim3(256), 0, s, n, m, \
                     p, p1, L, ldl, R1, ldr1, R2e, ldr2e, part, g.tiles_m, g.tiles_p,          \
                     g.rows_per_split)
    if (g.tm == 112 && g.tp == 112)  // seven waves, one 16-row stripe of 7 blocks each
      hipLaunchKernelGGL((gram_partial_kernel<T, 112, 112, 7, 1>), dim3(grid), dim3(kWave * 7), 0,
                         s, n, m, p, p1, L, ldl, R1, ldr1, R2e, ldr2e, part, g.tiles_m, g.tiles_p,
                         g.rows_per_split);
    else if (g.tm == 128 && g.tp == 128) LOBPCG_GRAM_LAUNCH(128, 128, 2);
    else if (g.tm == 128 && g.tp == 64) LOBPCG_GRAM_LAUNCH(128, 64, 2);
    else if (g.tm == 64 && g.tp == 128) LOBPCG_GRAM_LAUNCH(64, 128, 2);
    else if (g.tm == 64 && g.tp == 64) LOBPCG_GRAM_LAUNCH(64, 64, 2);
    else if (g.tm == 128 && g.tp == 112) LOBPCG_GRAM_LAUNCH(128, 112, 4);
    else if (g.tm == 112 && g.tp == 128) LOBPCG_GRAM_LAUNCH(112, 128, 1);
    else if (g.tm == 112 && g.tp == 64) LOBPCG_GRAM_LAUNCH(112, 64, 1);
    else LOBPCG_GRAM_LAUNCH(64, 112, 4);
#undef LOBPCG_GRAM_LAUNCH
    LOBPCG_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL(gram_reduce_kernel<double>, dim3(blocks_for((int64_t)m * p)), dim3(256), 0, s,
                     m, p, p1, nsplit, part, G1, c1, G2 ? G2 : G1, c2, ldg, mirror_rows);
  LOBPCG_HIP(hipGetLastError());
}
}  // namespace

template <typename T>
void launch_gram(int64_t n, int m, int p, int p1, const T* L, int64_t ldl, const T* R1,
                 int64_t ldr1, const T* R2, int64_t ldr2, double* G1, int c1, double* G2, int c2,
                 int64_t ldg, int mirror_rows, void* work, hipStream_t s) {
  if (m == 0 || p == 0) return;
  launch_gram_plan<T>(gram_plan(n, m, p, sizeof(T) == 4), n, m, p, p1, L, ldl, R1, ldr1, R2, ldr2,
                      G1, c1, G2, c2,
                      ldg, mirror_rows, work, s);
}

// ------------------------------------------------------------------ Gram without allocation
// The split-K partial tiles of lobpcg_gram_noalloc live in this fixed device
// array (one per GPU, held until the process ends) instead of a caller's
// workspace.  In host code the name is only a stand-in: kernels get the
// device address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[kGramScratchBytes / sizeof(double)];

namespace {
std::mutex g_scratch_mu;
std::vector<void*> g_scratch_ptr;  // per device ordinal
}  // namespace

void* gram_scratch_address() {
  int dev = 0;
  LOBPCG_HIP(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize(dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      throw Error(LOBPCG_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") +
                                      hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

template <typename T>
void launch_gram_noalloc(int64_t n, int m, int p, int p1, const T* L, int64_t ldl, const T* R1,
                         int64_t ldr1, const T* R2, int64_t ldr2, double* G1, int c1, double* G2,
                         int c2, int64_t ldg, int mirror_rows, hipStream_t s) {
  if (m == 0 || p == 0) return;
  const int64_t tile_bytes = (int64_t)m * p * (int64_t)sizeof(double);
  LOBPCG_CHECK(tile_bytes <= kGramScratchBytes, LOBPCG_ERR_ARG,
               "lobpcg_gram_noalloc: m * p * 8 = " + std::to_string(tile_bytes) +
                   " bytes exceeds the fixed scratch of " + std::to_string(kGramScratchBytes) +
                   " bytes");
  // the launch of lobpcg_gram, with the split count capped so that the
  // partial tiles fit the scratch (fewer, longer row ranges)
  GramPlan g = gram_plan(n, m, p, sizeof(T) == 4);
  const int64_t max_split = kGramScratchBytes / tile_bytes;
  if (g.nsplit > max_split) {
    int64_t rps = (n + max_split - 1) / max_split;
    rps = round_up(std::max<int64_t>(rps, kKB), kKB);
    g.nsplit = (int)std::max<int64_t>(1, (n + rps - 1) / rps);
    g.rows_per_split = rps;
  }
  launch_gram_plan<T>(g, n, m, p, p1, L, ldl, R1, ldr1, R2, ldr2, G1, c1, G2, c2, ldg,
                      mirror_rows, gram_scratch_address(), s);
}

int64_t gram_workspace_bound(int64_t n, int m, int p, bool fp32) {
  // nsplit <= max(1, target / tiles) and m * p <= tiles * kGramTM * kGramTP;
  // in FP32 also nsplit <= ceil(n / kGramFp32MaxRows) for any m' <= m, p' <= p.
  const int64_t row_splits = fp32 ? std::max<int64_t>(1, (n + kGramFp32MaxRows - 1) / kGramFp32MaxRows) : 1;
  return 8 * std::max<int64_t>((int64_t)kGramTargetBlocks * kGramTM * kGramTP,
                               (int64_t)m * p * row_splits);
}

template <typename T>
void launch_update(int64_t n, int K, int N, const T* S, int64_t lds, const double* C, int64_t ldc,
                   double alpha, double beta, T* Y, int64_t ldy, hipStream_t s) {
  if (n == 0 || N == 0) return;
  // the column tile (128, 112 or 64 wide) that pads N least; ties to the wider
  auto padded = [N](int t) { return (N + t - 1) / t * t; };
  int tn = kUpdTN;
  if (padded(112) < padded(tn)) tn = 112;
  if (padded(64) < padded(tn)) tn = 64;
  const int tiles_n = (N + tn - 1) / tn;
  const int64_t tiles_r = (n + kUpdTM - 1) / kUpdTM;
  const int64_t grid = tiles_r * tiles_n;
  LOBPCG_CHECK(grid < (int64_t)1 << 31, LOBPCG_ERR_ARG, "update grid too large");
  // 2 x 2 waves for 128- and 64-wide tiles; 4 x 1 (32 rows x 112 columns each) for 112.
  // FP64 with 112- or 64-wide tiles takes the LDS-DMA kernel where its layout holds.
  if constexpr (sizeof(T) == 8) {
    const bool dma = (tn == 112 || tn == 64) && K >= 2 && K % 2 == 0 && lds % 2 == 0 &&
                     reinterpret_cast<uintptr_t>(S) % 16 == 0;
    if (dma) {
      if (tn == 112)
        hipLaunchKernelGGL((update_dma_kernel<112, 4>), dim3((unsigned)grid), dim3(256), 0, s, n,
                           K, N, (const double*)S, lds, C, ldc, alpha, beta != 0.0 ? 1 : 0,
                           (double*)Y, ldy, tiles_n);
      else
        hipLaunchKernelGGL((update_dma_kernel<64, 2>), dim3((unsigned)grid), dim3(256), 0, s, n,
                           K, N, (const double*)S, lds, C, ldc, alpha, beta != 0.0 ? 1 : 0,
                           (double*)Y, ldy, tiles_n);
      LOBPCG_HIP(hipGetLastError());
      return;
    }
  }
  if (tn == 64)
    hipLaunchKernelGGL((update_kernel<T, 64, 2>), dim3((unsigned)grid), dim3(256), 0, s, n, K, N,
                       S, lds, C, ldc, (T)alpha, beta != 0.0 ? 1 : 0, Y, ldy, tiles_n);
  else if (tn == 112)
    hipLaunchKernelGGL((update_kernel<T, 112, 4>), dim3((unsigned)grid), dim3(256), 0, s, n, K, N,
                       S, lds, C, ldc, (T)alpha, beta != 0.0 ? 1 : 0, Y, ldy, tiles_n);
  else
    hipLaunchKernelGGL((update_kernel<T, kUpdTN, 2>), dim3((unsigned)grid), dim3(256), 0, s, n, K,
                       N, S, lds, C, ldc, (T)alpha, beta != 0.0 ? 1 : 0, Y, ldy, tiles_n);
  LOBPCG_HIP(hipGetLastError());
}

int64_t residual_workspace_bytes(int64_t n, int nx) {
  const int64_t nb = std::max<int64_t>(1, (n + kResRows - 1) / kResRows);
  return 2 * nb * (int64_t)std::max(nx, 1) * (int64_t)sizeof(double);
}

template <typename T>
void launch_residual(int64_t n, int nx, const T* AX, int64_t ldax, const T* BX, int64_t ldbx,
                     const T* X, int64_t ldx, const double* theta, const double* dinv, T* W,
                     int64_t ldw, double normA, double normB, double tol, double* rho,
                     int32_t* n_c, void* work, hipStream_t s) {
  if (nx == 0) return;
  const int64_t nb = std::max<int64_t>(1, (n + kResRows - 1) / kResRows);
  double* part_r = static_cast<double*>(work);
  double* part_x = part_r + nb * nx;
  hipLaunchKernelGGL((residual_kernel<T>), dim3((unsigned)nb, (unsigned)((nx + 63) / 64)),
                     dim3(256), 0, s, n, nx, AX, ldax, BX, ldbx, X, ldx, theta, dinv, W, ldw,
                     part_r, part_x);
  LOBPCG_HIP(hipGetLastError());
  hipLaunchKernelGGL(residual_rho_kernel, dim3((unsigned)nx), dim3(256), 0, s, nx, (int)nb, part_r,
                     part_x, theta, normA, normB, rho);
  hipLaunchKernelGGL(residual_nc_kernel, dim3(1), dim3(256), 0, s, nx, rho, theta, tol, n_c);
  LOBPCG_HIP(hipGetLastError());
}

template <typename P>
void launch_gram_reduce(int m, int p, int p1, int nparts, const P* part, double* G1, int c1,
                        double* G2, int c2, int64_t ldg, int mirror_rows, hipStream_t s) {
  if (m == 0 || p == 0) return;
  hipLaunchKernelGGL(gram_reduce_kernel<P>, dim3(blocks_for((int64_t)m * p)), dim3(256), 0, s, m,
                     p, p1, nparts, part, G1, c1, G2 ? G2 : G1, c2, ldg, mirror_rows);
  LOBPCG_HIP(hipGetLastError());
}
template void launch_gram_reduce<double>(int, int, int, int, const double*, double*, int, double*,
                                         int, int64_t, int, hipStream_t);
template void launch_gram_reduce<float>(int, int, int, int, const float*, double*, int, double*,
                                        int, int64_t, int, hipStream_t);

int64_t spmm_residual_workspace_bytes(int64_t n, int nx) {
  const int64_t nb = std::max<int64_t>(1, (n + kSpmmRowsPerBlock - 1) / kSpmmRowsPerBlock);
  return 2 * nb * (int64_t)std::max(nx, 1) * (int64_t)sizeof(double);
}

template <typename T>
void launch_spmm_residual(int64_t n, const int64_t* rowptr, const int32_t* colind,
                          const T* vals, const T* X, int64_t ldx, int nx, const double* theta,
                          const double* dinv, T* W, int64_t ldw, T* AX, int64_t ldax,
                          double normA, double tol, double* rho, int32_t* n_c, void* work,
                          hipStream_t s) {
  if (nx == 0 || n == 0) return;
  const int64_t nb = (n + kSpmmRowsPerBlock - 1) / kSpmmRowsPerBlock;
  LOBPCG_CHECK(nb < (int64_t)1 << 31, LOBPCG_ERR_ARG, "fused residual grid too large");
  double* part_r = static_cast<double*>(work);
  double* part_x = part_r + nb * nx;
  const unsigned gx = (unsigned)nb;
  if (nx <= 64) {
    hipLaunchKernelGGL((spmm_residual_kernel<T, 1>), dim3(gx, 1), dim3(256), 0, s, n, rowptr,
                       colind, vals, X, ldx, nx, theta, dinv, W, ldw, AX, ldax, part_r, part_x);
  } else if (nx <= 128) {
    hipLaunchKernelGGL((spmm_residual_kernel<T, 2>), dim3(gx, 1), dim3(256), 0, s, n, rowptr,
                       colind, vals, X, ldx, nx, theta, dinv, W, ldw, AX, ldax, part_r, part_x);
  } else {
    const unsigned gy = (unsigned)((nx + 255) / 256);
    hipLaunchKernelGGL((spmm_residual_kernel<T, 4>), dim3(gx, gy), dim3(256), 0, s, n, rowptr,
                       colind, vals, X, ldx, nx, theta, dinv, W, ldw, AX, ldax, part_r, part_x);
  }
  LOBPCG_HIP(hipGetLastError());
  hipLaunchKernelGGL(residual_rho_kernel, dim3((unsigned)nx), dim3(256), 0, s, nx, (int)nb, part_r,
                     part_x, theta, normA, 1.0, rho);
  hipLaunchKernelGGL(residual_nc_kernel, dim3(1), dim3(256), 0, s, nx, rho, theta, tol, n_c);
  LOBPCG_HIP(hipGetLastError());
}

int64_t colsq_workspace_bytes(int64_t n, int ncols) {
  const int64_t nb = std::max<int64_t>(1, (n + kResRows - 1) / kResRows);
  return nb * (int64_t)std::max(ncols, 1) * (int64_t)sizeof(double);
}

template <typename T>
void launch_colsq(int64_t n, int ncols, const T* Y, int64_t ldy, double* out, void* work,
                  hipStream_t s) {
  if (ncols == 0) return;
  const int64_t nb = std::max<int64_t>(1, (n + kResRows - 1) / kResRows);
  double* part = static_cast<double*>(work);
  hipLaunchKernelGGL((colsq_kernel<T>), dim3((unsigned)nb, (unsigned)((ncols + 63) / 64)),
                     dim3(256), 0, s, n, ncols, Y, ldy, part);
  LOBPCG_HIP(hipGetLastError());
  hipLaunchKernelGGL(colsq_finish_kernel, dim3((unsigned)ncols), dim3(256), 0, s, ncols, (int)nb,
                     part, out);
  LOBPCG_HIP(hipGetLastError());
}

int64_t jacobi_workspace_bytes(int64_t n) { return (3 * n + 4) * (int64_t)sizeof(double); }

void launch_jacobi_setup(int64_t n, const int64_t* rowptr, const int32_t* colind,
                         const double* vals, double* dinv, void* work, hipStream_t s) {
  if (n == 0) return;
  double* diag = static_cast<double*>(work);
  double* margin = diag + n;
  double* absrow = margin + n;
  double* stats = absrow + n;
  hipLaunchKernelGGL(jacobi_rows_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, rowptr, colind,
                     vals, diag, margin, absrow);
  hipLaunchKernelGGL(jacobi_reduce_kernel, dim3(1), dim3(256), 0, s, n, diag, margin, absrow,
                     stats);
  hipLaunchKernelGGL(jacobi_finish_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, diag, stats,
                     dinv);
  LOBPCG_HIP(hipGetLastError());
}

template <typename Tin, typename Tout>
void launch_copy2d(int64_t n, int ncols, const Tin* src, int64_t lds, Tout* dst, int64_t ldd,
                   hipStream_t s) {
  if (n == 0 || ncols == 0) return;
  hipLaunchKernelGGL((copy2d_kernel<Tin, Tout>), dim3(blocks_for(n * ncols)), dim3(256), 0, s, n,
                     ncols, src, lds, dst, ldd);
  LOBPCG_HIP(hipGetLastError());
}

template <typename T>
void launch_copy2d_reverse(int64_t n, int ncols, const T* src, int64_t lds, T* dst, int64_t ldd,
                           hipStream_t s) {
  if (n == 0 || ncols == 0) return;
  hipLaunchKernelGGL((copy2d_reverse_kernel<T>), dim3(blocks_for(n * ncols)), dim3(256), 0, s, n,
                     ncols, src, lds, dst, ldd);
  LOBPCG_HIP(hipGetLastError());
}

void launch_gaussian(int64_t n, int ncols, double* dst, int64_t ldd, uint64_t seed,
                     uint32_t stream, hipStream_t s) {
  const int64_t pairs = (n * ncols + 1) / 2;
  if (pairs == 0) return;
  hipLaunchKernelGGL(gaussian_kernel, dim3(blocks_for(pairs)), dim3(256), 0, s, n, ncols, dst, ldd,
                     seed, stream);
  LOBPCG_HIP(hipGetLastError());
}

void launch_fill_implicit(int nx, int np, const double* theta, const double* theta_p,
                          int64_t ldtp, double* GA, double* GB, int64_t ldg, hipStream_t s) {
  const int m = nx + np;
  if (m == 0) return;
  hipLaunchKernelGGL(fill_implicit_kernel, dim3(blocks_for((int64_t)m * m)), dim3(256), 0, s, nx,
                     np, theta, theta_p, ldtp, GA, GB, ldg);
  LOBPCG_HIP(hipGetLastError());
}

void launch_diag_scale(int n, const double* G, int64_t ldg, double* d, double* Gout, int64_t ldo,
                       bool compute_d, hipStream_t s) {
  if (n == 0) return;
  if (compute_d)
    hipLaunchKernelGGL(diag_d_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, G, ldg, d);
  hipLaunchKernelGGL(diag_scale_kernel, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, s, n, G,
                     ldg, d, Gout, ldo);
  LOBPCG_HIP(hipGetLastError());
}

void launch_cond1_upper(int n, const double* R, const double* Rinv, int64_t ld, double* cond,
                        double* scratch, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(upper_colsum_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, R,
                     Rinv, ld, scratch);
  hipLaunchKernelGGL(cond1_max_kernel, dim3(1), dim3(256), 0, s, n, scratch, cond);
  LOBPCG_HIP(hipGetLastError());
}

void launch_zero_lower(int n, double* A, int64_t ld, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(zero_lower_kernel, dim3(blocks_for((int64_t)n * n)), dim3(256), 0, s, n, A,
                     ld);
  LOBPCG_HIP(hipGetLastError());
}

void launch_row_scale(int m, int n, const double* d, double* A, int64_t lda, hipStream_t s) {
  if (m == 0 || n == 0) return;
  hipLaunchKernelGGL(row_scale_kernel, dim3(blocks_for((int64_t)m * n)), dim3(256), 0, s, m, n, d,
                     A, lda);
  LOBPCG_HIP(hipGetLastError());
}

void launch_row_scale_copy(int m, int n, const double* d, const double* A, int64_t lda, double* B,
                           int64_t ldb, hipStream_t s) {
  if (m == 0 || n == 0) return;
  hipLaunchKernelGGL(row_scale_copy_kernel, dim3(blocks_for((int64_t)m * n)), dim3(256), 0, s, m, n,
                     d, A, lda, B, ldb);
  LOBPCG_HIP(hipGetLastError());
}

void launch_col_scale(int m, int n, const double* A, int64_t lda, const double* theta, int mode,
                      double* B, int64_t ldb, hipStream_t s) {
  if (m == 0 || n == 0) return;
  hipLaunchKernelGGL(col_scale_kernel, dim3(blocks_for((int64_t)m * n)), dim3(256), 0, s, m, n, A,
                     lda, theta, mode, B, ldb);
  LOBPCG_HIP(hipGetLastError());
}

void launch_symmetrize(int n, double* A, int64_t lda, hipStream_t s) {
  if (n == 0) return;
  const int nt = (n + kSymTile - 1) / kSymTile;
  hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)(nt * (nt + 1) / 2)), dim3(256), 0, s, n, A,
                     lda);
  LOBPCG_HIP(hipGetLastError());
}

void launch_set_identity(int m, int n, double* A, int64_t lda, hipStream_t s) {
  if (m == 0 || n == 0) return;
  hipLaunchKernelGGL(set_identity_kernel, dim3(blocks_for((int64_t)m * n)), dim3(256), 0, s, m, n,
                     A, lda);
  LOBPCG_HIP(hipGetLastError());
}

void launch_negate(int n, const double* x, double* y, hipStream_t s) {
  if (n == 0) return;
  hipLaunchKernelGGL(negate_kernel, dim3(blocks_for(n)), dim3(256), 0, s, n, x, y);
  LOBPCG_HIP(hipGetLastError());
}

void launch_svqb_theta(int n, double* theta, double tau, int drop, double* scale, int32_t* info,
                       hipStream_t s) {
  hipLaunchKernelGGL(svqb_theta_kernel, dim3(1), dim3(256), 0, s, n, theta, tau, drop, scale, info);
  LOBPCG_HIP(hipGetLastError());
}

void launch_fro_minus_identity(int n, const double* A, int64_t lda, double* out, hipStream_t s) {
  hipLaunchKernelGGL(fro_kernel, dim3(1), dim3(256), 0, s, n, n, A, lda, 1, out);
  LOBPCG_HIP(hipGetLastError());
}

void launch_fro(int m, int n, const double* A, int64_t lda, double* out, hipStream_t s) {
  hipLaunchKernelGGL(fro_kernel, dim3(1), dim3(256), 0, s, m, n, A, lda, 0, out);
  LOBPCG_HIP(hipGetLastError());
}

void launch_sytrd_lower(int n, double* A, int64_t lda, double* d, double* e, double* tau,
                        hipStream_t s) {
  LOBPCG_CHECK(n >= 1 && n <= kTrdMaxN, LOBPCG_ERR_ARG, "sytrd: n out of range");
  if (n == 1) {
    LOBPCG_HIP(hipMemcpyAsync(d, A, sizeof(double), hipMemcpyDeviceToDevice, s));
    return;
  }
  if (lda % 2 == 0 && reinterpret_cast<uintptr_t>(A) % 16 == 0 &&
      lda * n * (int64_t)sizeof(double) <= INT32_MAX)
    hipLaunchKernelGGL(sytrd_lower_kernel<true>, dim3(1), dim3(kTrdThreads), 0, s, n, A, lda, d, e,
                       tau);
  else
    hipLaunchKernelGGL(sytrd_lower_kernel<false>, dim3(1), dim3(kTrdThreads), 0, s, n, A, lda, d, e,
                       tau);
  LOBPCG_HIP(hipGetLastError());
}

int sytrd_max_n() { return kTrdMaxN; }

bool geqrf_orgqr_fits(int m, int k) { return m >= 1 && m <= kQrMaxM && k >= 1 && k <= kQrCols && k <= m; }

void launch_geqrf_orgqr(int m, int k, double* M, int64_t ldm, hipStream_t s) {
  LOBPCG_CHECK(geqrf_orgqr_fits(m, k) && ldm >= m, LOBPCG_ERR_ARG, "geqrf_orgqr: sizes out of range");
  hipLaunchKernelGGL(geqrf_orgqr_kernel, dim3(1), dim3(kQrThreads), 0, s, m, k, M, ldm);
  LOBPCG_HIP(hipGetLastError());
}

void launch_ormtr_lower(int n, const double* A, int64_t lda, const double* tau, double* Z,
                        int64_t ldz, hipStream_t s) {
  LOBPCG_CHECK(n >= 1 && n <= kTrdMaxN, LOBPCG_ERR_ARG, "ormtr: n out of range");
  if (n < 2) return;
  const unsigned grid = (unsigned)((n + kOrmCols - 1) / kOrmCols);
  hipLaunchKernelGGL(ormtr_lower_kernel, dim3(grid), dim3(kOrmThreads), 0, s, n, A, lda, tau, Z,
                     ldz);
  LOBPCG_HIP(hipGetLastError());
}

void launch_sqrt_sum(int n, const double* v, double* out, hipStream_t s) {
  hipLaunchKernelGGL(sqrt_sum_kernel, dim3(1), dim3(256), 0, s, n, v, out);
  LOBPCG_HIP(hipGetLastError());
}

// ---- explicit instantiations
#define LOBPCG_INST(T)                                                                          \
  template void launch_spmm<T>(int64_t, const int64_t*, const int32_t*, const T*, const T*,    \
                               int64_t, T*, int64_t, int, hipStream_t);                         \
  template void launch_gram<T>(int64_t, int, int, int, const T*, int64_t, const T*, int64_t,   \
                               const T*, int64_t, double*, int, double*, int, int64_t, int,     \
                               void*, hipStream_t);                                             \
  template void launch_gram_noalloc<T>(int64_t, int, int, int, const T*, int64_t, const T*,    \
                                       int64_t, const T*, int64_t, double*, int, double*, int,  \
                                       int64_t, int, hipStream_t);                              \
  template void launch_update<T>(int64_t, int, int, const T*, int64_t, const double*, int64_t, \
                                 double, double, T*, int64_t, hipStream_t);                     \
  template void launch_residual<T>(int64_t, int, const T*, int64_t, const T*, int64_t,         \
                                   const T*, int64_t, const double*, const double*, T*,         \
                                   int64_t, double, double, double, double*, int32_t*, void*,   \
                                   hipStream_t);                                                \
  template void launch_colsq<T>(int64_t, int, const T*, int64_t, double*, void*, hipStream_t); \
  template void launch_spmm_residual<T>(int64_t, const int64_t*, const int32_t*, const T*,     \
                                        const T*, int64_t, int, const double*, const double*,  \
                                        T*, int64_t, T*, int64_t, double, double, double*,     \
                                        int32_t*, void*, hipStream_t);                          \
  template void launch_copy2d_reverse<T>(int64_t, int, const T*, int64_t, T*, int64_t,         \
                                         hipStream_t);
LOBPCG_INST(double)
LOBPCG_INST(float)
template void launch_copy2d<double, double>(int64_t, int, const double*, int64_t, double*, int64_t,
                                            hipStream_t);
template void launch_copy2d<double, float>(int64_t, int, const double*, int64_t, float*, int64_t,
                                           hipStream_t);
template void launch_copy2d<float, double>(int64_t, int, const float*, int64_t, double*, int64_t,
                                           hipStream_t);
template void launch_copy2d<float, float>(int64_t, int, const float*, int64_t, float*, int64_t,
                                          hipStream_t);

}  // namespace lobpcg
