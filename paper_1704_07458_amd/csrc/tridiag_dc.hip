// Divide and conquer for the symmetric tridiagonal eigenproblem T = Z diag(lam) Z^T
// (the step after the Householder tridiagonalisation of the projected matrix).
//
// Cuppen's tear: T = diag(T1, T2) + |b| w w^T with b = e[mid-1], w = e_{mid-1} +
// sign(b) e_mid, so T1's last and T2's first diagonal entries lose |b|.  A
// merge solves D + rho z z^T (D, Q from the halves, z = Q^T w / sqrt 2, rho = 2|b|)
// with LAPACK-style deflation (tiny rho |z_i|, and close pairs rotated until one
// z component vanishes), the secular equation 1 + rho sum z_i^2 / (d_i - lam) = 0
// solved root by root in the variable shifted to the nearer pole
// (so d_i - lam keeps full relative accuracy), z recomputed from the computed
// roots (Gu and Eisenstat) so that the eigenvectors z_i / (d_i - lam_j) are
// orthogonal to working precision, and one GEMM Q U per merge.  Leaves (at
// most kDcLeaf rows) use the implicit QL algorithm.
//
// The recursion tree depends only on n: node idx of level l (root level 0)
// covers the range obtained by halving [0, n) l times along the bits of idx
// (mid = (lo + hi) / 2), and all leaves sit at the same depth.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <cmath>
#include <string>

#include "small_gemm.hpp"
#include "tridiag_dc.hpp"
#include "wave.hpp"

#include "common.hpp"

namespace lobpcg {
namespace {

constexpr int kWave = 64;
constexpr int kDcLeaf = 16;
constexpr int kDcMaxN = 512;
constexpr int kDcThreads = 256;
constexpr int kDcQlIter = 60;
constexpr int kDcBisect = 128;

__device__ __forceinline__ void dc_range(int n, int level, int idx, int& lo, int& hi) {
  lo = 0;
  hi = n;
  for (int l = level - 1; l >= 0; --l) {
    const int mid = (lo + hi) / 2;
    if ((idx >> l) & 1)
      lo = mid;
    else
      hi = mid;
  }
}

__device__ __forceinline__ double dc_wave_sum(double v) { return wave64_sum(v); }

// ---------------------------------------------------------------- leaves
// One wave per leaf: the implicit QL algorithm with Wilkinson's shift on the
// leaf's tridiagonal block (the Bowdler-Martin-Reinsch-Wilkinson scheme).
// The leaf first takes the tears of the merges above it: every leaf boundary
// inside [0, n) is the split point mid of one merge, which removes |e[mid - 1]|
// from d[mid - 1] and d[mid] (so each d entry loses at most one such term).
// A leaf whose entries (d, its e and the two e at its boundaries) are not all
// finite is solved as the zero block instead, writes zeros over its own e and
// over a non-finite boundary e, and raises *fail to 2: every value the merges
// read is then finite (their ranks and orderings stay defined).
// Every lane runs the scalar recurrence on (d, e) in LDS with identical
// values; lane k applies each plane rotation to row k of the eigenvector
// block.  An off-diagonal e_i is negligible once |e_i| <= eps (|d_i| +
// |d_{i+1}|); at most kDcQlIter sweeps per eigenvalue (convergence is cubic,
// a few sweeps are the rule).  Writes lam[lo:hi) ascending and the leaf block
// Z[lo:hi, lo:hi).
// d and e stay in registers, lane k holding d_k and e_k: a uniform index is
// read with readlane and written with a lane select, so the scalar recurrence
// never waits on LDS.
__device__ __forceinline__ double dc_lane_get(double v, int i) {
  const int lo32 = __builtin_amdgcn_readlane(__double2loint(v), i);
  const int hi32 = __builtin_amdgcn_readlane(__double2hiint(v), i);
  return __hiloint2double(hi32, lo32);
}

__global__ __launch_bounds__(kWave) void dc_leaf_kernel(int n, int depth, const double* d,
                                                         double* e, double* lam,
                                                         double* __restrict__ Z, int64_t ldz,
                                                         int* __restrict__ fail) {
  __shared__ double V[kDcLeaf][kDcLeaf + 1];  // V[row][col]
  __shared__ double dl[kDcLeaf];
  __shared__ int perm[kDcLeaf];
  const int lane = threadIdx.x;
  constexpr double eps = 2.220446049250313e-16;
  int lo, hi;
  dc_range(n, depth, blockIdx.x, lo, hi);
  const int m = hi - lo;
  for (int q = lane; q < kDcLeaf * kDcLeaf; q += kWave) V[q / kDcLeaf][q % kDcLeaf] = (q / kDcLeaf == q % kDcLeaf) ? 1.0 : 0.0;
  const double din = lane < m ? d[lo + lane] : 0.0;
  const double ein = lane < m - 1 ? e[lo + lane] : 0.0;
  const double el = lo > 0 ? e[lo - 1] : 0.0;
  const double er = hi < n ? e[hi - 1] : 0.0;
  const bool bad = __ballot(!isfinite(din) || !isfinite(ein)) != 0 || !isfinite(el) ||
                   !isfinite(er);
  double dv = 0.0, ev = 0.0;
  if (!bad) {
    dv = din;
    ev = ein;
    if (lane == 0 && lo > 0) dv -= fabs(el);
    if (lane == m - 1 && hi < n) dv -= fabs(er);
  } else {
    if (lane < m - 1) e[lo + lane] = 0.0;
    if (lane == 0) {
      if (!isfinite(el)) e[lo - 1] = 0.0;
      if (!isfinite(er)) e[hi - 1] = 0.0;
      atomicMax(fail, 2);
    }
  }
  // scale by a power of two (exact) so that every entry is below 1 in magnitude
  double amax = fmax(fabs(dv), fabs(ev));
  for (int off = kWave / 2; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off, kWave));
  int ex = 0;
  if (amax > 0.0 && amax < INFINITY) frexp(amax, &ex);
  dv = ldexp(dv, -ex);
  ev = ldexp(ev, -ex);
  __syncthreads();
  bool stalled = false;
  for (int l = 0; l < m; ++l) {
    int it = 0;
    for (; it < kDcQlIter; ++it) {
      // first negligible e_mm at or after l (a wave-wide test)
      const bool neg = !(lane >= l && lane < m - 1) ||
                       fabs(ev) <= eps * (fabs(dv) + fabs(__shfl_down(dv, 1, kWave)));
      const unsigned long long mask = __ballot(neg && lane >= l) | (1ull << (m - 1));
      const int mm = __builtin_ctzll(mask >> l) + l;
      if (mm == l) break;
      // Wilkinson shift from the leading 2 x 2 block, as an offset g
      const double dl0 = dc_lane_get(dv, l), el0 = dc_lane_get(ev, l);
      double g = (dc_lane_get(dv, l + 1) - dl0) / (2.0 * el0);
      double r = hypot(g, 1.0);
      g = dc_lane_get(dv, mm) - dl0 + el0 / (g + copysign(r, g));
      double sn = 1.0, cs = 1.0, p = 0.0;
      bool split = false;
      double di1 = dc_lane_get(dv, mm);  // d_{i+1} for i = mm - 1
      for (int i = mm - 1; i >= l; --i) {
        const double ei = dc_lane_get(ev, i), di = dc_lane_get(dv, i);
        const double f = sn * ei, b = cs * ei;
        r = hypot(f, g);
        if (lane == i + 1) ev = r;
        if (r == 0.0) {  // the rotation underflowed: the block splits at i + 1
          if (lane == i + 1) dv = di1 - p;
          if (lane == mm) ev = 0.0;
          split = true;
          break;
        }
        const double rinv = 1.0 / r;
        sn = f * rinv;
        cs = g * rinv;
        g = di1 - p;
        r = (di - g) * sn + 2.0 * cs * b;
        p = sn * r;
        if (lane == i + 1) dv = g + p;
        g = cs * r - b;
        di1 = di;
        if (lane < m) {
          const double zi = V[lane][i], zi1 = V[lane][i + 1];
          V[lane][i + 1] = sn * zi + cs * zi1;
          V[lane][i] = cs * zi - sn * zi1;
        }
      }
      if (split) continue;
      if (lane == l) {
        dv -= p;
        ev = g;
      }
      if (lane == mm) ev = 0.0;
    }
    stalled = stalled || it == kDcQlIter;
  }
  // a leaf that did not converge within kDcQlIter sweeps per eigenvalue is
  // reported (its values are not trusted by the caller)
  if (stalled && lane == 0) atomicMax(fail, 1);
  if (lane < m) dl[lane] = ldexp(dv, ex);
  __syncthreads();
  // ascending order (rank sort, ties by index)
  if (lane < m) {
    const double w = dl[lane];
    int rank = 0;
    for (int j = 0; j < m; ++j) rank += (dl[j] < w || (dl[j] == w && j < lane)) ? 1 : 0;
    perm[rank] = lane;
  }
  __syncthreads();
  for (int q = lane; q < m * m; q += kWave) {
    const int r = q % m, k = q / m;
    Z[(int64_t)(lo + k) * ldz + lo + r] = V[r][perm[k]];
  }
  if (lane < m) lam[lo + lane] = dl[perm[lane]];
}

// Per-node bookkeeping in the int workspace (offsets from the base):
//   [node]                 K (values entering the secular equation)
//   [kNrot + node]         number of rotations
//   [kOrd + lo + k]        position of sorted slot k ([kept ascending | deflated])
//   [kSrc + lo + k]        child column of position k (< n1: left, else right)
//   [kRp / kRi + lo + r]   rotation r acts on positions (p, i), in order
//   [kPerm + lo + k]       slot of the k-th smallest eigenvalue of the node
// and in the double workspace: rotation cosines / sines at [lo + r] and [kDcMaxN + lo + r].
constexpr int kNrot = 64, kOrd = 128, kSrc = kOrd + kDcMaxN, kRp = kSrc + kDcMaxN,
              kRi = kRp + kDcMaxN, kPerm = kRi + kDcMaxN, kDcInts = kPerm + kDcMaxN;
static_assert(kDcInts <= 4096, "int workspace");

// Bit sets over a node's positions, 64 per word: the highest set position
// below i (or -1), the lowest at or above from (or -1), the count below i.
__device__ __forceinline__ int dc_prev_set(const unsigned long long* w, int i) {
  int q = i >> 6;
  unsigned long long b = w[q] & ((1ull << (i & 63)) - 1);
  while (b == 0) {
    if (--q < 0) return -1;
    b = w[q];
  }
  return (q << 6) + 63 - __builtin_clzll(b);
}

__device__ __forceinline__ int dc_next_set(const unsigned long long* w, int nw, int from) {
  int q = from >> 6;
  if (q >= nw) return -1;
  unsigned long long b = w[q] & (~0ull << (from & 63));
  while (b == 0) {
    if (++q >= nw) return -1;
    b = w[q];
  }
  return (q << 6) + __builtin_ctzll(b);
}

__device__ __forceinline__ int dc_count_below(const unsigned long long* w, int i) {
  int c = 0;
  const int q = i >> 6;
  for (int k = 0; k < q; ++k) c += __popcll(w[k]);
  return c + __popcll(w[q] & ((1ull << (i & 63)) - 1));
}

// ---------------------------------------------------------------- merge: prepare
// One workgroup per node: sorted d and z, deflation, the order [kept ascending
// | deflated], the rotation list, rho of the kept set.
// Close pairs are a scan over the survivors of the small-z test, each against
// the previous survivor as the earlier steps of the scan left it.  A survivor
// whose predecessor is unchanged is tested against the predecessor's own
// values, so those tests run in parallel first (bit set cw); the sequential
// pass then starts at each flagged survivor and follows the chain of rotations
// from it while the next survivor is close to the rotated value: the same
// tests on the same values, in the same order, as a scan over every survivor.
// The order: when the kept values ascend in position order (checked), a kept
// entry's rank is the number of kept entries before it and a deflated one's K
// plus the deflated entries before it (counts of bits); otherwise the ranks
// come from comparisons with every entry.
__global__ __launch_bounds__(kDcThreads) void dc_prepare_kernel(
    int n, int level, const double* __restrict__ e, const double* __restrict__ lam,
    const double* __restrict__ Z, int64_t ldz, double* __restrict__ dsort,
    double* __restrict__ zsort, int* __restrict__ iw, double* __restrict__ rw,
    double* __restrict__ rhoK) {
  __shared__ double ds[kDcMaxN], zs[kDcMaxN], lm[kDcMaxN];
  __shared__ int src[kDcMaxN], defl[kDcMaxN];
  __shared__ int K_s;
  __shared__ double rho_s, znorm_s;
  __shared__ double wmax[2][kDcThreads / kWave];
  __shared__ unsigned long long sw[kDcMaxN / 64], cw[kDcMaxN / 64], kw[kDcMaxN / 64];
  __shared__ int unsorted;
  const int t = threadIdx.x;
  const int lane = t % kWave, wv = t / kWave;
  const int node = blockIdx.x;
  int lo, hi;
  dc_range(n, level, node, lo, hi);
  const int mid = (lo + hi) / 2;
  const int m = hi - lo, n1 = mid - lo, n2 = hi - mid;
  const double b = e[mid - 1];
  const double rho = 2.0 * fabs(b);
  const double sg = b < 0.0 ? -1.0 : 1.0;
  const double rs2 = 0.70710678118654752440;
  for (int i = t; i < m; i += kDcThreads) lm[i] = lam[lo + i];
  __syncthreads();
  // merge the two ascending eigenvalue lists (ties: left half first)
  for (int i = t; i < m; i += kDcThreads) {
    double di, zi;
    int rank;
    if (i < n1) {
      di = lm[i];
      zi = Z[(int64_t)(lo + i) * ldz + (mid - 1)] * rs2;
      int a = 0, c = n2;  // number of right entries < di
      while (a < c) {
        const int h = (a + c) / 2;
        if (lm[n1 + h] < di) a = h + 1; else c = h;
      }
      rank = i + a;
    } else {
      const int i2 = i - n1;
      di = lm[n1 + i2];
      zi = sg * Z[(int64_t)(mid + i2) * ldz + mid] * rs2;
      int a = 0, c = n1;  // number of left entries <= di
      while (a < c) {
        const int h = (a + c) / 2;
        if (lm[h] <= di) a = h + 1; else c = h;
      }
      rank = i2 + a;
    }
    ds[rank] = di;
    zs[rank] = zi;
    src[rank] = i;
  }
  __syncthreads();
  {
    double dmax = 0.0, zmax = 0.0;
    for (int i = t; i < m; i += kDcThreads) {
      dmax = fmax(dmax, fabs(ds[i]));
      zmax = fmax(zmax, fabs(zs[i]));
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
      dmax = fmax(dmax, __shfl_xor(dmax, off, kWave));
      zmax = fmax(zmax, __shfl_xor(zmax, off, kWave));
    }
    if (t % kWave == 0) {
      wmax[0][t / kWave] = dmax;
      wmax[1][t / kWave] = zmax;
    }
  }
  __syncthreads();
  double dmax = 0.0, zmax = 0.0;
  for (int w = 0; w < kDcThreads / kWave; ++w) {
    dmax = fmax(dmax, wmax[0][w]);
    zmax = fmax(zmax, wmax[1][w]);
  }
  const double tol = 8.0 * 2.220446049250313e-16 * fmax(dmax, zmax);
  // deflation of tiny rho |z_i|, in parallel
  for (int i = t; i < m; i += kDcThreads) defl[i] = (rho * fabs(zs[i]) <= tol) ? 1 : 0;
  __syncthreads();
  const int nw = (m + 63) / 64;
  for (int w = wv; w < nw; w += kDcThreads / kWave) {
    const int i = 64 * w + lane;
    const unsigned long long b = __ballot(i < m && !defl[i]);
    if (lane == 0) sw[w] = b;
  }
  __syncthreads();
  // |dt c s| <= tol (c^2 + s^2) is |dt c s| / (c^2 + s^2) <= tol without the
  // square root and divisions (the rotation is formed only for a close pair)
  for (int w = wv; w < nw; w += kDcThreads / kWave) {
    const int i = 64 * w + lane;
    bool close = false;
    if (i < m && !defl[i]) {
      const int p = dc_prev_set(sw, i);
      if (p >= 0) {
        const double di = ds[i], zi = zs[i], pd = ds[p], pz = zs[p];
        close = fabs((di - pd) * zi * pz) <= tol * fma(zi, zi, pz * pz);
      }
    }
    const unsigned long long b = __ballot(close);
    if (lane == 0) cw[w] = b;
  }
  __syncthreads();
  if (t == 0) {
    int nrot = 0;
    int i = dc_next_set(cw, nw, 0);
    while (i >= 0) {
      int prev = dc_prev_set(sw, i);
      double pd = ds[prev], pz = zs[prev];
      for (;;) {
        const double di = ds[i], zi = zs[i];
        if (!(fabs((di - pd) * zi * pz) <= tol * fma(zi, zi, pz * pz))) break;
        const double tau = hypot(zi, pz);
        const double cc = zi / tau, ss = -pz / tau;
        const double dnew = pd * ss * ss + di * cc * cc;
        zs[i] = tau;
        zs[prev] = 0.0;
        ds[prev] = pd * cc * cc + di * ss * ss;
        ds[i] = dnew;
        defl[prev] = 1;
        iw[kRp + lo + nrot] = prev;
        iw[kRi + lo + nrot] = i;
        rw[lo + nrot] = cc;
        rw[kDcMaxN + lo + nrot] = ss;
        ++nrot;
        pd = dnew;
        pz = tau;
        prev = i;
        i = dc_next_set(sw, nw, i + 1);
        if (i < 0) break;
      }
      if (i < 0) break;
      i = dc_next_set(cw, nw, i + 1);
    }
    iw[kNrot + node] = nrot;
  }
  __syncthreads();
  // K and |z_kept|^2: per-thread partials, wave sums, then the waves in order
  {
    double zp = 0.0;
    int kc = 0;
    for (int i = t; i < m; i += kDcThreads)
      if (!defl[i]) {
        ++kc;
        zp = fma(zs[i], zs[i], zp);
      }
    zp = wave64_sum(zp);
    for (int off = kWave / 2; off > 0; off >>= 1) kc += __shfl_xor(kc, off, kWave);
    if (t % kWave == 0) {
      wmax[0][t / kWave] = zp;
      wmax[1][t / kWave] = (double)kc;
    }
  }
  __syncthreads();
  if (t == 0) {
    double zn = 0.0;
    int K = 0;
    for (int w = 0; w < kDcThreads / kWave; ++w) {
      zn += wmax[0][w];
      K += (int)wmax[1][w];
    }
    K_s = K;
    znorm_s = sqrt(zn);
    rho_s = rho * zn;
    iw[node] = K;
    rhoK[node] = rho * zn;
  }
  __syncthreads();
  const int K = K_s;
  for (int w = wv; w < nw; w += kDcThreads / kWave) {
    const int i = 64 * w + lane;
    const unsigned long long b = __ballot(i < m && !defl[i]);
    if (lane == 0) kw[w] = b;
  }
  if (t == 0) unsorted = 0;
  __syncthreads();
  for (int i = t; i < m; i += kDcThreads)
    if (!defl[i]) {
      const int p = dc_prev_set(kw, i);
      if (p >= 0 && ds[p] > ds[i]) unsorted = 1;
    }
  __syncthreads();
  const bool ascending = unsorted == 0;
  for (int i = t; i < m; i += kDcThreads) {
    // kept: the kept entries before it in (value, index) order; deflated: K
    // plus the deflated entries before it.  Without ascending kept values:
    // eight entries' reads in flight per step and branch-free counts (one LDS
    // round trip per eight entries).
    const double di = ds[i];
    const bool dfi = defl[i] != 0;
    int rank = 0;
    int j = 0;
    if (ascending) {
      const int kb = dc_count_below(kw, i);
      rank = dfi ? i - kb : kb;
      j = m;
    }
    for (; j + 8 <= m; j += 8) {
      double dj[8];
      int fj[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        dj[u] = ds[j + u];
        fj[u] = defl[j + u];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {  // bitwise logic: no short-circuit branches
        const int before = (int)(j + u < i), f = (int)(fj[u] != 0);
        const int lt = (int)(dj[u] < di), eq = (int)(dj[u] == di);
        rank += dfi ? (f & before) : ((1 - f) & (lt | (eq & before)));
      }
    }
    for (; j < m; ++j)
      rank += dfi ? ((defl[j] && j < i) ? 1 : 0)
                  : ((!defl[j] && (ds[j] < di || (ds[j] == di && j < i))) ? 1 : 0);
    if (dfi) rank += K;
    iw[kOrd + lo + rank] = i;
    dsort[lo + rank] = ds[i];
    if (rank < K) zsort[lo + rank] = zs[i] / znorm_s;
    iw[kSrc + lo + i] = src[i];
  }
}

// ---------------------------------------------------------------- merge: stage
// One workgroup per (node, position k): Qs[lo:hi, lo + k] = column src[k] of
// diag(Q1, Q2) (the other child's rows zero).
__device__ __forceinline__ void dc_stage(int bid, int n, int level, int mmax,
                                         const int* __restrict__ iw, const double* __restrict__ Z,
                                         double* __restrict__ Qs, int64_t ldz) {
  const int node = bid / mmax, k = bid % mmax;
  int lo, hi;
  dc_range(n, level, node, lo, hi);
  const int m = hi - lo, n1 = (lo + hi) / 2 - lo;
  if (k >= m) return;
  // child column sidx sits at global column lo + sidx (the right child's
  // columns follow the left child's)
  const int sidx = iw[kSrc + lo + k];
  const bool left = sidx < n1;
  const double* zc = Z + (int64_t)(lo + sidx) * ldz;
  double* qc = Qs + (int64_t)(lo + k) * ldz + lo;
  for (int r = threadIdx.x; r < m; r += kDcThreads)
    qc[r] = (left ? r < n1 : r >= n1) ? zc[lo + r] : 0.0;
}

// ---------------------------------------------------------------- merge: rotate
// One thread per (node, row): the deflation rotations, in order, on the row.
__device__ __forceinline__ void dc_rotate(int bid, int n, int level, int rblocks,
                                          const int* __restrict__ iw,
                                          const double* __restrict__ rw, double* __restrict__ Qs,
                                          int64_t ldz) {
  const int node = bid / rblocks;
  const int r = (bid % rblocks) * kDcThreads + threadIdx.x;
  int lo, hi;
  dc_range(n, level, node, lo, hi);
  if (r >= hi - lo) return;
  const int nrot = iw[kNrot + node];
  double* row = Qs + lo + r;
  for (int k = 0; k < nrot; ++k) {
    const int p = iw[kRp + lo + k], i = iw[kRi + lo + k];
    const double cc = rw[lo + k], ss = rw[kDcMaxN + lo + k];
    double* qp = row + (int64_t)(lo + p) * ldz;
    double* qi = row + (int64_t)(lo + i) * ldz;
    const double a = *qp, c = *qi;
    *qp = cc * a + ss * c;
    *qi = -ss * a + cc * c;
  }
}

// ---------------------------------------------------------------- merge: secular roots
// One wave per (node, root j < K), lanes sharing the sums over the kept set.
// The root is located in the variable tau shifted to the nearer pole, by Newton
// steps on -tau f(tau) safeguarded by the bracketing interval.  Each lane keeps
// its share of d and z (entries lane, lane + 64, ...) in registers for the
// whole iteration, so a step is arithmetic and wave sums only.
// lamk[lo + j] = root j;  Dl[lo + i, lo + j] = d_i - root_j.
__device__ __forceinline__ void dc_secular(int bid, int n, int level, int rblocks,
                                           const double* __restrict__ dsort,
                                           const double* __restrict__ zsort,
                                           const int* __restrict__ iw,
                                           const double* __restrict__ rhoK,
                                           double* __restrict__ lamk, double* __restrict__ Dl,
                                           int64_t ldz) {
  const int node = bid / rblocks;
  const int lane = threadIdx.x % kWave;
  const int j = (bid % rblocks) * (kDcThreads / kWave) + threadIdx.x / kWave;
  int lo, hi;
  dc_range(n, level, node, lo, hi);
  const int K = iw[node];
  if (j >= K) return;
  const double rho = rhoK[node];
  const double* dd = dsort + lo;
  const double* zz = zsort + lo;
  constexpr int kPer = kDcMaxN / kWave;
  double dr[kPer], zr[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = lane + u * kWave;
    dr[u] = i < K ? dd[i] : 0.0;
    zr[u] = i < K ? zz[i] : 0.0;
  }
  int o;
  double a, c;
  if (j < K - 1) {
    const double half = 0.5 * (dd[j + 1] - dd[j]);
    const double dj = dd[j];
    double f = 0.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u)
      if (lane + u * kWave < K) f += zr[u] * zr[u] / ((dr[u] - dj) - half);
    f = 1.0 + rho * dc_wave_sum(f);
    if (f >= 0.0) {
      o = j;
      a = 0.0;
      c = half;
    } else {
      o = j + 1;
      a = -half;
      c = 0.0;
    }
  } else {
    o = K - 1;
    a = 0.0;
    c = rho;  // |z| = 1: the last root lies within rho of d_K
  }
  const double dor = dd[o];
  double tau = 0.5 * (a + c);
  for (int it = 0; it < kDcBisect; ++it) {
    double f = 0.0, fp = 0.0, fa = 0.0;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      if (lane + u * kWave >= K) continue;
      const double q = zr[u] / ((dr[u] - dor) - tau);
      f = fma(zr[u], q, f);
      fp = fma(q, q, fp);
      fa += fabs(zr[u] * q);
    }
    f = 1.0 + rho * dc_wave_sum(f);
    fp = rho * dc_wave_sum(fp);
    fa = 1.0 + rho * dc_wave_sum(fa);
    // |f| at the level of its own rounding error: tau is as good as it gets
    if (fabs(f) <= 8.0 * 2.220446049250313e-16 * fa) break;
    if (f > 0.0)
      c = tau;
    else
      a = tau;
    // Newton on F(tau) = -tau f(tau), which has no pole at the origin (the
    // pole the root is nearest to): tau <- tau^2 f' / (f + tau f'); bisection
    // when the step leaves the bracket
    const double den = f + tau * fp;
    double nt = tau * tau * fp / den;
    if (!(nt > a && nt < c)) nt = 0.5 * (a + c);
    if (nt == tau || nt == a || nt == c) break;
    if (fabs(nt - tau) <= 2.220446049250313e-16 * fabs(nt)) {
      tau = nt;
      break;
    }
    tau = nt;
  }
  if (lane == 0) lamk[lo + j] = dor + tau;
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int i = lane + u * kWave;
    if (i < K) Dl[(int64_t)(lo + j) * ldz + lo + i] = (dr[u] - dor) - tau;
  }
}

// ---------------------------------------------------------------- merge: zhat
// One thread per (node, i < K): z recomputed from the roots (Gu-Eisenstat),
// zhat_i^2 = (root_i - d_i) / rho  prod_{j != i} (root_j - d_i) / (d_j - d_i).
__device__ __forceinline__ void dc_zhat(int bid, int n, int level, int rblocks,
                                        const double* __restrict__ dsort,
                                        const double* __restrict__ zsort,
                                        const int* __restrict__ iw,
                                        const double* __restrict__ rhoK,
                                        const double* __restrict__ Dl, double* __restrict__ zh,
                                        int64_t ldz) {
  const int node = bid / rblocks;
  const int i = (bid % rblocks) * kDcThreads + threadIdx.x;
  int lo, hi;
  dc_range(n, level, node, lo, hi);
  const int K = iw[node];
  if (i >= K) return;
  const double* dd = dsort + lo;
  const double* dcol = Dl + (int64_t)lo * ldz + lo + i;  // Dl(i, j) = dcol[j ldz]
  const double di = dd[i];
  double prod = -dcol[(int64_t)i * ldz] / rhoK[node];
  int j = 0;
  for (; j + 8 <= K; j += 8) {  // batches of independent loads, then the products
    double v[8], w[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      v[u] = dcol[(int64_t)(j + u) * ldz];
      w[u] = dd[j + u];
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (j + u != i) prod *= -v[u] / (w[u] - di);
  }
  for (; j < K; ++j)
    if (j != i) prod *= -dcol[(int64_t)j * ldz] / (dd[j] - di);
  zh[lo + i] = copysign(sqrt(fmax(prod, 0.0)), zsort[lo + i]);
}

// ---------------------------------------------------------------- merge: vectors
// One workgroup (one wave) per (node, column j < m): U(:, j) = zhat / (d - root_j)
// normalised (zero below row K), and the GEMM operand G(:, j) = kept column j of
// Qs (zero for j >= K).
__global__ __launch_bounds__(kWave) void dc_vectors_kernel(int n, int level, int mmax,
                                                           const int* __restrict__ iw,
                                                           const double* __restrict__ zh,
                                                           const double* __restrict__ Qs,
                                                           double* __restrict__ Dl,
                                                           double* __restrict__ G, int64_t ldz) {
  const int node = blockIdx.x / mmax, j = blockIdx.x % mmax;
  const int lane = threadIdx.x;
  int lo, hi;
  dc_range(n, level, node, lo, hi);
  const int m = hi - lo;
  if (j >= m) return;
  const int K = iw[node];
  double* gc = G + (int64_t)(lo + j) * ldz + lo;
  if (j < K) {
    const double* qc = Qs + (int64_t)(lo + iw[kOrd + lo + j]) * ldz + lo;
    for (int r = lane; r < m; r += kWave) gc[r] = qc[r];
    double* u = Dl + (int64_t)(lo + j) * ldz + lo;
    double s = 0.0;
    for (int i = lane; i < K; i += kWave) {
      const double v = zh[lo + i] / u[i];
      u[i] = v;
      s = fma(v, v, s);
    }
    const double inv = 1.0 / sqrt(dc_wave_sum(s));
    for (int i = lane; i < m; i += kWave) u[i] = i < K ? u[i] * inv : 0.0;
  } else {
    for (int r = lane; r < m; r += kWave) gc[r] = 0.0;
  }
}

// ---------------------------------------------------------------- merge: order
// One workgroup per node: ascending order of the node's eigenvalues (kept
// roots, then deflated d), lam[lo:hi) and the slot of each.
__device__ __forceinline__ void dc_order(int bid, int n, int level, int* __restrict__ iw,
                                         const double* __restrict__ lamk,
                                         const double* __restrict__ dsort,
                                         double* __restrict__ lam) {
  __shared__ double w[kDcMaxN];
  const int t = threadIdx.x;
  const int node = bid;
  int lo, hi;
  dc_range(n, level, node, lo, hi);
  const int m = hi - lo;
  const int K = iw[node];
  for (int i = t; i < m; i += kDcThreads) w[i] = i < K ? lamk[lo + i] : dsort[lo + i];
  __syncthreads();
  for (int i = t; i < m; i += kDcThreads) {
    // rank in (value, index) order, eight entries' reads in flight per step
    const double wi = w[i];
    int rank = 0;
    int j = 0;
    for (; j + 8 <= m; j += 8) {
      double wj[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) wj[u] = w[j + u];
#pragma unroll
      for (int u = 0; u < 8; ++u)
        rank += (int)(wj[u] < wi) | ((int)(wj[u] == wi) & (int)(j + u < i));
    }
    for (; j < m; ++j) rank += (w[j] < wi || (w[j] == wi && j < i)) ? 1 : 0;
    iw[kPerm + lo + rank] = i;
    lam[lo + rank] = wi;
  }
}

// ---------------------------------------------------------------- merge: fused launches
// Steps of a merge level that depend only on earlier launches share one
// launch (each workgroup takes one step's block; the branch is uniform over
// the workgroup).  After prepare: the secular roots (blocks [0, nodes sblocks))
// and the staging of the child columns.  After those: the order of the node's
// eigenvalues (one block per node), zhat, and the deflation rotations of the
// staged columns.  The steps of one launch read nothing another writes.
__global__ __launch_bounds__(kDcThreads) void dc_secular_stage_kernel(
    int n, int level, int sblocks, int mmax, const double* __restrict__ dsort,
    const double* __restrict__ zsort, const int* __restrict__ iw,
    const double* __restrict__ rhoK, double* __restrict__ lamk, double* __restrict__ Dl,
    const double* __restrict__ Z, double* __restrict__ Qs, int64_t ldz) {
  const int nsec = (1 << level) * sblocks;
  const int bid = (int)blockIdx.x;
  if (bid < nsec)
    dc_secular(bid, n, level, sblocks, dsort, zsort, iw, rhoK, lamk, Dl, ldz);
  else
    dc_stage(bid - nsec, n, level, mmax, iw, Z, Qs, ldz);
}

__global__ __launch_bounds__(kDcThreads) void dc_order_zhat_rotate_kernel(
    int n, int level, int rblocks, int* __restrict__ iw, const double* __restrict__ lamk,
    const double* __restrict__ dsort, double* __restrict__ lam, const double* __restrict__ zsort,
    const double* __restrict__ rhoK, const double* __restrict__ Dl, double* __restrict__ zh,
    const double* __restrict__ rw, double* __restrict__ Qs, int64_t ldz) {
  const int nodes = 1 << level;
  const int bid = (int)blockIdx.x;
  if (bid < nodes)
    dc_order(bid, n, level, iw, lamk, dsort, lam);
  else if (bid < nodes + nodes * rblocks)
    dc_zhat(bid - nodes, n, level, rblocks, dsort, zsort, iw, rhoK, Dl, zh, ldz);
  else
    dc_rotate(bid - nodes - nodes * rblocks, n, level, rblocks, iw, rw, Qs, ldz);
}

// ---------------------------------------------------------------- merge: scatter
// One workgroup per (node, output column k): Z[lo:hi, lo + k] from the GEMM
// output (kept slots) or the staged deflated column.
__global__ __launch_bounds__(kDcThreads) void dc_scatter_kernel(int n, int level, int mmax,
                                                                const int* __restrict__ iw,
                                                                const double* __restrict__ Y,
                                                                const double* __restrict__ Qs,
                                                                double* __restrict__ Z,
                                                                int64_t ldz) {
  const int node = blockIdx.x / mmax, k = blockIdx.x % mmax;
  int lo, hi;
  dc_range(n, level, node, lo, hi);
  const int m = hi - lo;
  if (k >= m) return;
  const int K = iw[node];
  const int slot = iw[kPerm + lo + k];
  const double* sc = slot < K ? Y + (int64_t)(lo + slot) * ldz + lo
                              : Qs + (int64_t)(lo + iw[kOrd + lo + slot]) * ldz + lo;
  double* zc = Z + (int64_t)(lo + k) * ldz + lo;
  for (int r = threadIdx.x; r < m; r += kDcThreads) zc[r] = sc[r];
}

inline void dc_check(rocblas_status st, const char* what) {
  if (st != rocblas_status_success)
    throw Error(LOBPCG_ERR_HIP, std::string(what) + ": " + rocblas_status_to_string(st));
}

inline unsigned dc_blocks(int64_t total, int per) { return (unsigned)((total + per - 1) / per); }

}  // namespace

int tridiag_dc_max_n() { return kDcMaxN; }
int tridiag_dc_int_workspace() { return kDcInts; }

void tridiag_dc(int n, double* d, const double* e, double* lam, double* Z, int64_t ldz,
                double* Qs, double* Dl, double* G, double* Y, double* vec4, int* iw, double* rw,
                double* rhoK, int* fail, rocblas_handle h, hipStream_t s) {
  LOBPCG_CHECK(n >= 1 && n <= kDcMaxN && ldz >= n, LOBPCG_ERR_ARG, "tridiag_dc: bad sizes");
  int depth = 0;
  while (((n + (1 << depth) - 1) >> depth) > kDcLeaf) ++depth;
  double* dsort = vec4;
  double* zsort = vec4 + n;
  double* lamk = vec4 + 2 * n;
  double* zh = vec4 + 3 * n;
  hipLaunchKernelGGL(dc_leaf_kernel, dim3(1u << depth), dim3(kWave), 0, s, n, depth, d,
                     const_cast<double*>(e), lam, Z, ldz, fail);
  LOBPCG_HIP(hipGetLastError());
  for (int level = depth - 1; level >= 0; --level) {
    const int nodes = 1 << level;
    const int mmax = (n + nodes - 1) / nodes;
    const int rb = (int)dc_blocks(mmax, kDcThreads);
    const int sb = (int)dc_blocks(mmax, kDcThreads / kWave);
    hipLaunchKernelGGL(dc_prepare_kernel, dim3(nodes), dim3(kDcThreads), 0, s, n, level, e, lam,
                       Z, ldz, dsort, zsort, iw, rw, rhoK);
    hipLaunchKernelGGL(dc_secular_stage_kernel, dim3(nodes * (sb + mmax)), dim3(kDcThreads), 0, s,
                       n, level, sb, mmax, dsort, zsort, iw, rhoK, lamk, Dl, Z, Qs, ldz);
    hipLaunchKernelGGL(dc_order_zhat_rotate_kernel, dim3(nodes * (1 + 2 * rb)), dim3(kDcThreads), 0,
                       s, n, level, rb, iw, lamk, dsort, lam, zsort, rhoK, Dl, zh, rw, Qs, ldz);
    hipLaunchKernelGGL(dc_vectors_kernel, dim3(nodes * mmax), dim3(kWave), 0, s, n, level, mmax,
                       iw, zh, Qs, Dl, G, ldz);
    LOBPCG_HIP(hipGetLastError());
    // Y = G U over each node's full block: G is zero beyond the kept columns
    // and U zero below the kept rows (the kept count is known on the device
    // only); all nodes of the level in one launch
    int offs[kSmallGemmBatch], dims[kSmallGemmBatch];
    for (int node = 0; node < nodes; ++node) {
      int lo = 0, hi = n;
      for (int l = level - 1; l >= 0; --l) {
        const int mid = (lo + hi) / 2;
        if ((node >> l) & 1) lo = mid; else hi = mid;
      }
      offs[node] = lo;
      dims[node] = hi - lo;
    }
    small_dgemm_diag_batch(nodes, offs, dims, G, ldz, Dl, ldz, Y, ldz, s);
    hipLaunchKernelGGL(dc_scatter_kernel, dim3(nodes * mmax), dim3(kDcThreads), 0, s, n, level,
                       mmax, iw, Y, Qs, Z, ldz);
    LOBPCG_HIP(hipGetLastError());
  }
}

}  // namespace lobpcg
