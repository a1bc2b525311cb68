// Dense symmetric eigensolver for the small matrices of the method: the
// Gram blocks H_B^T H_B and H_W^T H_W (whose eigenpairs give the cores of
// the exponentials and the spectral shift) and the Rayleigh-Ritz matrices
// of block Lanczos.  One workgroup per matrix (batched over the grid),
// float64 throughout.
//
//   1. Householder reduction to tridiagonal form T = Q^T A Q.  The working
//      matrix lives in LDS when it fits (n <= kLdsMax; two barriers per
//      reflector), else in global memory (three barriers per reflector).
//   2. Eigenvalues of T by Sturm-count multisection: groups of g threads
//      probe 4 g points per step; the count uses the three-term recurrence
//      of the leading principal minors (no divisions) on T scaled by a power
//      of two, rescaled by powers of 2 every four steps.
//   3. Eigenvectors of T by inverse iteration, one thread per eigenvalue
//      (LU with partial pivoting of T - lambda I, two solves with
//      overflow-safe rescaling), then orthonormalisation inside clusters of
//      close eigenvalues (Cholesky QR twice by the whole workgroup, or
//      classical Gram-Schmidt twice for very large clusters).  By default
//      the clusters are tight (gaps up to 1e-8 ||T||) and a first-order
//      correction of the whole block, Z <- Z (I - (Z^T Z - I) / 2), then
//      removes the small overlaps between clusters.
//   4. Back-transformation by the stored reflectors, applied straight to the
//      eigenvectors of T: held in registers (LDS path) or in LDS panels with
//      the reflectors staged in blocks (global path).
#include <cstdio>
#include <type_traits>

#include "common.h"

namespace eda {

namespace {

constexpr int SYEV_NMAX = 2048;
constexpr int kLdsMax = 128;      // largest n whose working matrix is kept in LDS
constexpr int kLdsDoubles = 160 * 1024 / 8;  // all of a CU's LDS (global path)
constexpr int kClusterMax = 64;   // clusters up to this size use Cholesky QR

template <int NT>
__device__ __forceinline__ double blk_sum(double v, double* red) {
  constexpr int NW = NT / 64;
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NW; ++w) s += red[w];
  return s;
}

template <int NT>
__device__ __forceinline__ double blk_max(double v, double* red) {
  constexpr int NW = NT / 64;
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < NW; ++w) s = fmax(s, red[w]);
  return s;
}

template <int NT>
__device__ __forceinline__ double blk_min(double v, double* red) {
  constexpr int NW = NT / 64;
  for (int m = 32; m >= 1; m >>= 1) v = fmin(v, __shfl_xor(v, m));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < NW; ++w) s = fmin(s, red[w]);
  return s;
}

// sum_k a[k*sa] b[k*sb], k < len: loads issued U at a time into four
// accumulators (fixed order, so the result is reproducible).
template <int U>
__device__ __forceinline__ double dot_pipe(const double* __restrict__ a, int64_t sa,
                                           const double* __restrict__ b, int64_t sb, int len) {
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  int k = 0;
  for (; k + U <= len; k += U) {
    double x[U], y[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x[u] = a[(int64_t)(k + u) * sa];
      y[u] = b[(int64_t)(k + u) * sb];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) acc[u & 3] += x[u] * y[u];
  }
  for (; k < len; ++k) acc[0] += a[(int64_t)k * sa] * b[(int64_t)k * sb];
  return (acc[0] + acc[1]) + (acc[2] + acc[3]);
}

__device__ __forceinline__ uint64_t hash64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

// Counts for K points at once (K independent recurrences interleaved), for
// a T scaled so that |d_k|, e_k^2 and |x| are at most 4: a minor grows by at
// most 8x per step, so the power-of-two rescaling is checked every four
// steps (thresholds 2^+-600).  A zero minor becomes -2^-60 times its
// predecessor: tiny, of the opposite sign, counted as a change.
template <int K>
__device__ __forceinline__ void sturm_counts(int n, const double* __restrict__ D,
                                             const double* __restrict__ E2, const double* x,
                                             int* cnt) {
  double pm2[K], pm1[K];
#pragma unroll
  for (int q = 0; q < K; ++q) {
    pm2[q] = 1.0;
    pm1[q] = D[0] - x[q];
    if (pm1[q] == 0.0) pm1[q] = -0x1.0p-60;
    cnt[q] = (pm1[q] < 0.0);
  }
  int k = 1;
  for (; k + 3 < n; k += 4) {
    double dk[4], fk[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      dk[u] = D[k + u];
      fk[u] = E2[k - 1 + u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int q = 0; q < K; ++q) {
        double p = fma(dk[u] - x[q], pm1[q], -fk[u] * pm2[q]);
        p = (p == 0.0) ? -0x1.0p-60 * pm1[q] : p;
        cnt[q] += ((p < 0.0) != (pm1[q] < 0.0));
        pm2[q] = pm1[q];
        pm1[q] = p;
      }
    }
#pragma unroll
    for (int q = 0; q < K; ++q) {
      const double mx = fmax(fabs(pm1[q]), fabs(pm2[q]));
      const double f = (mx > 0x1.0p600) ? 0x1.0p-600 : ((mx < 0x1.0p-600) ? 0x1.0p600 : 1.0);
      pm1[q] *= f;
      pm2[q] *= f;
    }
  }
  for (; k < n; ++k) {
    const double dv = D[k], fv = E2[k - 1];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      double p = fma(dv - x[q], pm1[q], -fv * pm2[q]);
      p = (p == 0.0) ? -0x1.0p-60 * pm1[q] : p;
      cnt[q] += ((p < 0.0) != (pm1[q] < 0.0));
      pm2[q] = pm1[q];
      pm1[q] = p;
    }
  }
}

// LU factorisation with partial pivoting of T - lam I (T tridiagonal: diagonal
// D, off-diagonal ee).  Stored per position k with stride NT: 1/U(k,k),
// U(k,k+1), U(k,k+2), the multiplier and the interchange flag.
template <int NT>
__device__ __forceinline__ void tri_factor(int n, const double* __restrict__ D, const double* __restrict__ ee,
                           double lam, double tiny, double* __restrict__ lu, int64_t nmax) {
  double* U1 = lu;
  double* U2 = lu + nmax * NT;
  double* U3 = lu + 2 * nmax * NT;
  double* Lm = lu + 3 * nmax * NT;
  double* Pv = lu + 4 * nmax * NT;
#define LU(arr, k) arr[(int64_t)(k) * NT]
  double p = D[0] - lam;
  double qv = (n > 1) ? ee[0] : 0.0;
  double rv = 0.0;
  for (int k = 0; k < n - 1; ++k) {
    const double ek = ee[k];
    const double an = D[k + 1] - lam;
    const double en = (k + 1 < n - 1) ? ee[k + 1] : 0.0;  // (D and ee are in LDS)
    if (fabs(p) >= fabs(ek)) {
      if (fabs(p) < tiny) p = (p < 0.0) ? -tiny : tiny;
      const double inv = 1.0 / p;
      const double l = ek * inv;
      LU(U1, k) = inv;
      LU(U2, k) = qv;
      LU(U3, k) = rv;
      LU(Lm, k) = l;
      LU(Pv, k) = 0.0;
      p = an - l * qv;
      qv = en - l * rv;
    } else {
      const double inv = 1.0 / ek;
      const double l = p * inv;
      LU(U1, k) = inv;
      LU(U2, k) = an;
      LU(U3, k) = en;
      LU(Lm, k) = l;
      LU(Pv, k) = 1.0;
      p = qv - l * an;
      qv = rv - l * en;
    }
    rv = 0.0;
  }
  if (fabs(p) < tiny) p = (p < 0.0) ? -tiny : tiny;
  LU(U1, n - 1) = 1.0 / p;
  LU(U2, n - 1) = 0.0;
  LU(U3, n - 1) = 0.0;
#undef LU
}

// Solve (T - lam I) x = y in place (y with stride ys).  The back substitution
// rescales the whole system whenever the solution grows past 2^300, so chains
// of tiny pivots (split matrices, multiple eigenvalues) cannot overflow.
template <int NT>
__device__ __forceinline__ void tri_solve(int n, const double* __restrict__ lu, int64_t nmax,
                          double* __restrict__ y, int64_t ys) {
  const double* U1 = lu;
  const double* U2 = lu + nmax * NT;
  const double* U3 = lu + 2 * nmax * NT;
  const double* Lm = lu + 3 * nmax * NT;
  const double* Pv = lu + 4 * nmax * NT;
#define LU(arr, k) arr[(int64_t)(k) * NT]
#define YV(k) y[(int64_t)(k) * ys]
  // Loads are issued eight steps at a time: each original entry is read
  // once, before the step that overwrites it.
  double carry = YV(0);
  int k = 0;
  for (; k + 8 <= n - 1; k += 8) {
    double yb[8], pv[8], lm[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      yb[q] = YV(k + 1 + q);
      pv[q] = LU(Pv, k + q);
      lm[q] = LU(Lm, k + q);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double a = carry, b = yb[q];
      if (pv[q] != 0.0) {
        const double t = a;
        a = b;
        b = t;
      }
      YV(k + q) = a;
      carry = b - lm[q] * a;
    }
  }
  for (; k < n - 1; ++k) {
    double a = carry, b = YV(k + 1);
    if (LU(Pv, k) != 0.0) {
      const double t = a;
      a = b;
      b = t;
    }
    YV(k) = a;
    carry = b - LU(Lm, k) * a;
  }
  YV(n - 1) = carry;
  const double big = 0x1.0p300, small = 0x1.0p-300;
  double x2 = 0.0, x1 = 0.0;  // x[k+2], x[k+1]
  k = n - 1;
  for (; k >= 7; k -= 8) {
    double yv[8], u1[8], u2[8], u3[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      yv[q] = YV(k - q);
      u1[q] = LU(U1, k - q);
      u2[q] = LU(U2, k - q);
      u3[q] = LU(U3, k - q);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      double x = (yv[q] - u2[q] * x1 - u3[q] * x2) * u1[q];
      if (!(fabs(x) < big)) {
        for (int j = 0; j < n; ++j) YV(j) *= small;
#pragma unroll
        for (int r = 0; r < 8; ++r) yv[r] *= small;
        x1 *= small;
        x2 *= small;
        x = (yv[q] - u2[q] * x1 - u3[q] * x2) * u1[q];
      }
      YV(k - q) = x;
      x2 = x1;
      x1 = x;
    }
  }
  for (; k >= 0; --k) {
    double x = (YV(k) - LU(U2, k) * x1 - LU(U3, k) * x2) * LU(U1, k);
    if (!(fabs(x) < big)) {
      for (int j = 0; j < n; ++j) YV(j) *= small;
      x1 *= small;
      x2 *= small;
      x = (YV(k) - LU(U2, k) * x1 - LU(U3, k) * x2) * LU(U1, k);
    }
    YV(k) = x;
    x2 = x1;
    x1 = x;
  }
#undef YV
#undef LU
}

__device__ __forceinline__ void random_start(int n, int i, double* y, int64_t ys) {
  for (int k = 0; k < n; ++k) {
    const uint64_t h = hash64(((uint64_t)(i + 1) << 32) ^ (uint64_t)k ^ 0x5bd1e995ull);
    y[(int64_t)k * ys] = ((double)(h >> 11) * 0x1.0p-53) * 2.0 - 1.0;
  }
}

// y / ||y||, one thread; loads in batches of 8 so that each batch costs one
// memory round trip (y lives in global memory).
__device__ __forceinline__ void normalize_serial(int n, double* y, int64_t ys) {
  double mx = 0.0;
  for (int k0 = 0; k0 < n; k0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (k0 + u < n) ? y[(int64_t)(k0 + u) * ys] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) mx = fmax(mx, fabs(v[u]));
  }
  const double inv = (mx > 0.0) ? 1.0 / mx : 1.0;
  double nrm = 0.0;
  for (int k0 = 0; k0 < n; k0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (k0 + u < n) ? y[(int64_t)(k0 + u) * ys] * inv : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u) nrm += v[u] * v[u];
  }
  const double sc = inv / sqrt(nrm);
  for (int k0 = 0; k0 < n; k0 += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (k0 + u < n) ? y[(int64_t)(k0 + u) * ys] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (k0 + u < n) y[(int64_t)(k0 + u) * ys] = v[u] * sc;
  }
}

// Orthogonality correction of the nv columns of Z (n x nv, row stride nv) by
// the whole workgroup: with E = Z^T Z - I, Z <- Z (I - E / 2), which leaves
// Z^T Z = I - 3 E^2 / 4 + O(E^3); repeated (at most three times) until
// max |E_ij| <= 16 u.  Meant for columns whose pairwise products are already
// small (inverse-iteration vectors of eigenvalues separated by g, which
// overlap by about u ||T|| / g): column j then moves by sum_i E_ij z_i, and
// its residual by about sum_i |E_ij| |lambda_i - lambda_j| = O(u ||T||).
// E lives in Eg (nv x nv), the updated block in Zn (n x nv) before it is
// copied back; both are global scratch.
template <int NT>
__device__ __forceinline__ void wg_orth_correct(int n, int nv, double* __restrict__ Z,
                                                double* __restrict__ Eg, double* __restrict__ Zn,
                                                double* red) {
  const int tid = threadIdx.x;
  const int nb4 = (nv + 3) >> 2, nr4 = (n + 3) >> 2;
  const int L = nb4 * (nb4 + 1) / 2;
  for (int pass = 0; pass < 3; ++pass) {
    double emax = 0.0;
    for (int p = tid; p < L; p += NT) {
      int bi = (int)((sqrt(8.0 * (double)p + 1.0) - 1.0) * 0.5);
      while ((bi + 1) * (bi + 2) / 2 <= p) ++bi;
      while (bi * (bi + 1) / 2 > p) --bi;
      const int bj = p - bi * (bi + 1) / 2;
      const int i0 = 4 * bi, j0 = 4 * bj;
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      for (int pos = 0; pos < n; ++pos) {
        const double* zr = Z + (int64_t)pos * nv;
        double zi[4], zj[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          zi[a] = (i0 + a < nv) ? zr[i0 + a] : 0.0;
          zj[a] = (j0 + a < nv) ? zr[j0 + a] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(zi[a], zj[b], acc[a][b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int i = i0 + a, j = j0 + b;
          if (i < nv && j <= i) {
            const double e = acc[a][b] - (i == j ? 1.0 : 0.0);
            Eg[(int64_t)i * nv + j] = e;
            Eg[(int64_t)j * nv + i] = e;
            emax = fmax(emax, fabs(e));
          }
        }
    }
    emax = blk_max<NT>(emax, red);  // its barriers publish E
    if (!(emax > 16.0 * 0x1.0p-53)) break;
    for (int p = tid; p < nr4 * nb4; p += NT) {
      const int r0 = 4 * (p / nb4), j0 = 4 * (p % nb4);
      double acc[4][4];
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;
      for (int q = 0; q < nv; ++q) {
        double zq[4], eq[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          zq[a] = (r0 + a < n) ? Z[(int64_t)(r0 + a) * nv + q] : 0.0;
          eq[a] = (j0 + a < nv) ? Eg[(int64_t)q * nv + j0 + a] : 0.0;
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) acc[a][b] = fma(zq[a], eq[b], acc[a][b]);
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int r = r0 + a, j = j0 + b;
          if (r < n && j < nv)
            Zn[(int64_t)r * nv + j] = fma(-0.5, acc[a][b], Z[(int64_t)r * nv + j]);
        }
    }
    __syncthreads();
    for (int e = tid; e < n * nv; e += NT) Z[e] = Zn[e];
    __syncthreads();
  }
}

__device__ void wave_normalize(int n, double* y, int64_t ys, int lane) {
  double mx = 0.0;
  for (int k = lane; k < n; k += 64) mx = fmax(mx, fabs(y[(int64_t)k * ys]));
  for (int m = 32; m >= 1; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m));
  const double inv = (mx > 0.0) ? 1.0 / mx : 1.0;
  double nrm = 0.0;
  for (int k = lane; k < n; k += 64) {
    const double v = y[(int64_t)k * ys] * inv;
    nrm += v * v;
  }
  nrm = wave_sum(nrm);
  const double sc = (nrm > 0.0) ? inv / sqrt(nrm) : 0.0;
  for (int k = lane; k < n; k += 64) y[(int64_t)k * ys] *= sc;
}

// Global work per matrix (doubles): A n^2, d/e/tau/lambda 4n, Z_T n^2,
// LU 5 n NT (+ n of slack).
__host__ __device__ inline int64_t syev_work_doubles(int64_t nmax, int nt) {
  return 5 * nmax + 2 * nmax * nmax + 5 * nmax * (int64_t)nt;
}

// LDS layout (doubles):
//   LDS path:    A [n (n+1)] | sv [n] | sw [n] | red [16] | Gc [syev_lds_gc(n)]
//                | Zt [n nvec] (when it fits)
//   global path: sv [n] | sw [n] | red [32] | stage [rest of the 160 KB]  (Gc = stage)
// LDS path: the cluster Gram matrices (Gc) take what the working matrix
// leaves of the 160 KB, at most kClusterMax^2 doubles (3680 at n = 128, so
// clusters of up to 60 vectors use Cholesky QR there); Gc also holds the
// wave partials of the tridiagonalisation (NW 128 + NW <= 1032 doubles).
__host__ __device__ inline int64_t syev_lds_gc(int64_t n) {
  const int64_t rest = kLdsDoubles - (n * (n + 1) + 2 * n + 32);
  const int64_t full = (int64_t)kClusterMax * kClusterMax;
  return rest < full ? rest : full;
}
__host__ __device__ inline int64_t syev_lds_doubles(int64_t n, bool lds_a) {
  return lds_a ? n * (n + 1) + 2 * n + 32 + syev_lds_gc(n) : kLdsDoubles;
}
// LDS path: the eigenvectors of T (n x nvec) follow when they fit in 160 KB.
inline int64_t syev_lds_alloc(int64_t nmax, int64_t nvmax, bool lds_a) {
  const int64_t base = syev_lds_doubles(nmax, lds_a);
  return (lds_a && base + nmax * nvmax <= kLdsDoubles) ? base + nmax * nvmax : base;
}

// Optional per-phase cycle counters (matrix 0 of each launch), for profiling.
__device__ unsigned long long g_syev_cycles[8];

#define SYEV_MARK(ph)                                                           \
  do {                                                                          \
    if (timing && q == 0 && tid == 0) {                                         \
      const unsigned long long now_ = clock64();                                \
      atomicAdd(&g_syev_cycles[ph], now_ - t_prev);                             \
      t_prev = now_;                                                            \
    }                                                                           \
  } while (0)

// Matrix q of the launch: given by sarr[q] when sarr is not null (any
// pointers, each with its own work area of syev_work_doubles(nmax, NT)),
// else at the strided positions below.
template <int NT>
__global__ __launch_bounds__(NT) void syev_kernel(const SyevArgs* __restrict__ sarr, int nfix,
                                                  const int* __restrict__ ns,
                                                  const double* __restrict__ Ain, int64_t lda_,
                                                  int64_t strideA, double* __restrict__ wout,
                                                  int64_t stridew, double* __restrict__ Zout,
                                                  int64_t ldz_, int64_t strideZ, int nvec_,
                                                  double* __restrict__ work, int64_t nmax,
                                                  int lds_a, int timing, double ctol_,
                                                  int64_t lds_cap) {
  constexpr int NW = NT / 64;
  constexpr int DU = NT > 512 ? 4 : 8;  // dot-product unroll within the register budget
  extern __shared__ double smem[];
  const int q = blockIdx.x;
  int n, nvec_req;
  double ctol_rel = ctol_;
  int64_t lda, ldz;
  const double* Aq;
  double *wq, *Zq, *wk;
  if (sarr != nullptr) {
    const SyevArgs a = sarr[q];
    n = (int)a.n;
    lda = a.lda;
    ldz = a.ldz;
    nvec_req = (int)a.nvec;
    ctol_rel = a.ctol;
    Aq = a.A;
    wq = a.w;
    Zq = a.Z;
    wk = a.work;
  } else {
    n = (ns != nullptr) ? ns[q] : nfix;
    lda = lda_;
    ldz = ldz_;
    nvec_req = nvec_;
    Aq = Ain + q * strideA;
    wq = wout + q * stridew;
    Zq = Zout + q * strideZ;
    wk = work + q * syev_work_doubles(nmax, NT);
  }
  if (n <= 0) return;
  const int nv = (nvec_req <= 0 || nvec_req > n) ? n : nvec_req;
  double* gA = wk;                   // n x n (global path)
  double* dd = gA + nmax * nmax;
  double* ee = dd + nmax;
  double* tau = ee + nmax;
  double* lamv = tau + nmax;
  double* ZtG = lamv + nmax;         // [pos][slot] (work area)
  double* lub = ZtG + nmax * nmax;   // LU arrays, [array][pos][thread]
  // [pos][slot] in LDS when the launch reserved n nv doubles past the rest
  double* ZtL = smem + syev_lds_doubles(nmax, true);
  const bool zt_lds = lds_a && syev_lds_doubles(nmax, true) + (int64_t)n * nv <= lds_cap;
  double *A, *sv, *sw, *red, *stage, *Gc;
  int64_t ldA;
  if (lds_a) {
    A = smem;
    ldA = nmax + 1;
    sv = smem + nmax * (nmax + 1);
    sw = sv + nmax;
    red = sw + nmax;
    Gc = red + 32;
    stage = nullptr;
  } else {
    A = gA;
    ldA = nmax;
    sv = smem;
    sw = sv + nmax;
    red = sw + nmax;
    stage = red + 32;
    Gc = stage;
  }
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const double eps = 0x1.0p-53;
  unsigned long long t_prev = clock64();

  // ---- 0. symmetrised working copy (lower triangle of the input) ---------
  for (int c = wid; c < n; c += NW)
    for (int r = lane; r < n; r += 64)
      A[r + (int64_t)c * ldA] = (r >= c) ? Aq[r + c * lda] : Aq[c + r * lda];
  __syncthreads();

  SYEV_MARK(0);
  // ---- 1. Householder tridiagonalisation ---------------------------------
  if (NT <= 512 && lds_a) {
    // Working matrix in LDS, two barriers per reflector.  Lane l of every
    // wave holds rows j+1+l and j+65+l of the trailing block; wave w takes
    // the columns j+1+w, j+1+w+NW, ...  The wave partials of A v (and of
    // v^T A v) meet in LDS at the first barrier; each thread then forms
    // w = tau A v - (tau^2 v^T A v / 2) v for its rows and applies the
    // rank-2 update to its columns, taking w of a column from the lane that
    // holds that row.  The norm of the next column below its subdiagonal is
    // summed by wave 0, which updates that column, so the next reflector
    // needs no further reduction.  Reflector j is scaled into column j of A
    // one step later, when nothing reads that column any more.
    double* const AL = smem;     // the same matrix, addressed as LDS
    double* pw = Gc;              // NW x 128 wave partials of A v
    double* dw = Gc + NW * 128;   // NW wave partials of v^T A v
    double* cn = red;             // next-column norms, alternating slots
    const int wsu = __builtin_amdgcn_readfirstlane(wid);  // wave index, known uniform
    if (wid == 0) {
      double s0 = 0.0;
      for (int r = 2 + lane; r < n; r += 64) s0 += AL[r] * AL[r];
      s0 = wave_sum(s0);
      if (lane == 0) cn[0] = s0;
    }
    __syncthreads();
    double scale_prev = 0.0;
    for (int j = 0; j < n - 2; ++j) {
      const double* col = AL + (int64_t)j * ldA;
      if (j > 0)
        for (int r = j + 1 + tid; r < n; r += NT) AL[r + (int64_t)(j - 1) * ldA] *= scale_prev;
      const double s = cn[j & 1];
      const double alpha = col[j + 1];
      double beta, tv, scale;
      if (s == 0.0) {
        tv = 0.0;
        beta = alpha;
        scale = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + s), alpha);
        tv = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      if (tid == 0) {
        dd[j] = col[j];
        ee[j] = beta;
        tau[j] = tv;
      }
      scale_prev = scale;
      const int r0 = j + 1 + lane, r1 = r0 + 64;
      if (tv == 0.0) {
        if (wid == 0) {
          const double* c1 = AL + (int64_t)(j + 1) * ldA;
          double s1 = 0.0;
          for (int r = j + 3 + lane; r < n; r += 64) s1 += c1[r] * c1[r];
          s1 = wave_sum(s1);
          if (lane == 0) cn[(j + 1) & 1] = s1;
        }
        __syncthreads();
        continue;
      }
      const double y0 = col[r0], y1 = col[r1];  // rows past n: in-range LDS, masked
      const double v0 = (r0 == j + 1) ? 1.0 : (r0 < n ? y0 * scale : 0.0);
      const double v1 = (r1 < n) ? y1 * scale : 0.0;
      // loads of four columns are issued together; rows past n read
      // in-range LDS and are masked
      double a0 = 0.0, a1 = 0.0;
      int c = j + 1 + wsu;
      for (; c + 3 * NW < n; c += 4 * NW) {
        double vc[4], x0[4], x1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int cu = c + u * NW;
          const double* ac = AL + (int64_t)cu * ldA;
          vc[u] = col[cu];
          x0[u] = ac[r0];
          x1[u] = ac[r1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) vc[u] = (c + u * NW == j + 1) ? 1.0 : vc[u] * scale;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a0 += (r0 < n ? x0[u] : 0.0) * vc[u];
          a1 += (r1 < n ? x1[u] : 0.0) * vc[u];
        }
      }
      for (; c < n; c += NW) {
        const double cv = col[c];
        const double* ac = AL + (int64_t)c * ldA;
        const double x0 = ac[r0], x1 = ac[r1];
        const double vc = (c == j + 1) ? 1.0 : cv * scale;
        a0 += (r0 < n ? x0 : 0.0) * vc;
        a1 += (r1 < n ? x1 : 0.0) * vc;
      }
      const double dsum = wave_sum(v0 * a0 + v1 * a1);
      pw[wid * 128 + lane] = a0;
      pw[wid * 128 + 64 + lane] = a1;
      if (lane == 0) dw[wid] = dsum;
      __syncthreads();
      double p0 = 0.0, p1 = 0.0, vav = 0.0;
      for (int w = 0; w < NW; ++w) {
        p0 += pw[w * 128 + lane];
        p1 += pw[w * 128 + 64 + lane];
        vav += dw[w];
      }
      const double K = 0.5 * tv * tv * vav;
      const double w0 = tv * p0 - K * v0, w1 = tv * p1 - K * v1;
      c = j + 1 + wsu;
      for (; c + 3 * NW < n; c += 4 * NW) {
        double vc[4], wc[4], x0[4], x1[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int cu = c + u * NW;
          const int lc = cu - (j + 1);
          const double* ac = AL + (int64_t)cu * ldA;
          vc[u] = col[cu];
          wc[u] = (lc < 64) ? readlane_f64(w0, lc) : readlane_f64(w1, lc - 64);
          x0[u] = ac[r0];
          x1[u] = ac[r1];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) vc[u] = (c + u * NW == j + 1) ? 1.0 : vc[u] * scale;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          double* ac = AL + (int64_t)(c + u * NW) * ldA;
          if (r0 < n) ac[r0] = x0[u] - (v0 * wc[u] + w0 * vc[u]);
          if (r1 < n) ac[r1] = x1[u] - (v1 * wc[u] + w1 * vc[u]);
        }
      }
      for (; c < n; c += NW) {
        const int lc = c - (j + 1);
        const double cv = col[c];
        const double wc = (lc < 64) ? readlane_f64(w0, lc) : readlane_f64(w1, lc - 64);
        double* ac = AL + (int64_t)c * ldA;
        const double x0 = ac[r0], x1 = ac[r1];
        const double vc = (c == j + 1) ? 1.0 : cv * scale;
        if (r0 < n) ac[r0] = x0 - (v0 * wc + w0 * vc);
        if (r1 < n) ac[r1] = x1 - (v1 * wc + w1 * vc);
      }
      if (wsu == 0) {  // wave 0 updated column j+1: its norm below row j+2
        const double* c1 = AL + (int64_t)(j + 1) * ldA;
        const double y0 = c1[r0], y1 = c1[r1];
        double nrm = (r0 >= j + 3 && r0 < n) ? y0 * y0 : 0.0;
        nrm += (r1 < n) ? y1 * y1 : 0.0;
        nrm = wave_sum(nrm);
        if (lane == 0) cn[(j + 1) & 1] = nrm;
      }
      __syncthreads();
    }
    if (n >= 3 && tid == 0) AL[(n - 1) + (int64_t)(n - 3) * ldA] *= scale_prev;
  } else {
    // Working matrix in global memory (L2-resident at these sizes), three
    // barriers per reflector.  v lives in LDS (sv); wave w forms the entries
    // p_r = (A v)_r of the rows r = j+1+w, j+1+w+NW, ... (lanes over the
    // column of A that equals row r), keeping p in sw and its share of
    // v^T A v in dw; the rank-2 update then takes w_c = tau p_c - K v_c on
    // the fly, waves over columns and lanes over rows, and wave 0 sums the
    // next column's norm while updating it.
    double* const AG = gA;
    double* dw = red + 2;  // NW <= 16 partials of v^T A v (red holds 16 + 2 doubles)
    double* cn = red;
    if (wid == 0) {
      double s0 = 0.0;
      for (int r = 2 + lane; r < n; r += 64) s0 += AG[r] * AG[r];
      s0 = wave_sum(s0);
      if (lane == 0) cn[0] = s0;
    }
    __syncthreads();
    for (int j = 0; j < n - 2; ++j) {
      double* col = AG + (int64_t)j * ldA;
      const double s = cn[j & 1];
      const double alpha = col[j + 1];
      double beta, tv, scale;
      if (s == 0.0) {
        tv = 0.0;
        beta = alpha;
        scale = 0.0;
      } else {
        beta = -copysign(sqrt(alpha * alpha + s), alpha);
        tv = (beta - alpha) / beta;
        scale = 1.0 / (alpha - beta);
      }
      if (tid == 0) {
        dd[j] = col[j];
        ee[j] = beta;
        tau[j] = tv;
      }
      if (tv == 0.0) {
        if (wid == 0) {
          const double* c1 = AG + (int64_t)(j + 1) * ldA;
          double s1 = 0.0;
          for (int r = j + 3 + lane; r < n; r += 64) s1 += c1[r] * c1[r];
          s1 = wave_sum(s1);
          if (lane == 0) cn[(j + 1) & 1] = s1;
        }
        __syncthreads();
        continue;
      }
      for (int r = j + 1 + tid; r < n; r += NT) {
        const double v = (r == j + 1) ? 1.0 : col[r] * scale;
        sv[r] = v;
        if (r >= j + 2) col[r] = v;  // reflector j, kept for the back-transformation
      }
      __syncthreads();
      // four rows per pass, their loads issued together
      double dpart = 0.0;
      for (int r0 = j + 1 + wid; r0 < n; r0 += 4 * NW) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int c = j + 1 + lane; c < n; c += 64) {
          const double vc = sv[c];
          double x[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int r = r0 + u * NW;
            x[u] = (r < n) ? AG[c + (int64_t)r * ldA] : 0.0;  // column r = row r
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] += x[u] * vc;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int r = r0 + u * NW;
          const double p = wave_sum(acc[u]);
          if (r < n) {
            dpart += sv[r] * p;
            if (lane == 0) sw[r] = p;
          }
        }
      }
      if (lane == 0) dw[wid] = dpart;
      __syncthreads();
      double vav = 0.0;
      for (int w = 0; w < NW; ++w) vav += dw[w];
      const double K = 0.5 * tv * tv * vav;
      // four columns per pass; each lane loads up to four of its rows of
      // them before storing any
      for (int c0 = j + 1 + wid; c0 < n; c0 += 4 * NW) {
        double vc[4], wc[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int c = c0 + u * NW;
          vc[u] = (c < n) ? sv[c] : 0.0;
          wc[u] = (c < n) ? tv * sw[c] - K * vc[u] : 0.0;
        }
        double nrm = 0.0;
        for (int rb = j + 1 + lane; rb < n; rb += 256) {
          double x[4][4], vr[4], wr[4];
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = rb + 64 * q;
            vr[q] = (r < n) ? sv[r] : 0.0;
            wr[q] = (r < n) ? tv * sw[r] - K * vr[q] : 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int c = c0 + u * NW;
              x[q][u] = (r < n && c < n) ? AG[r + (int64_t)c * ldA] : 0.0;
            }
          }
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int r = rb + 64 * q;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const int c = c0 + u * NW;
              if (r < n && c < n) {
                const double y = x[q][u] - (vr[q] * wc[u] + wr[q] * vc[u]);
                AG[r + (int64_t)c * ldA] = y;
                if (u == 0 && c == j + 1 && r >= j + 3) nrm += y * y;
              }
            }
          }
        }
        if (c0 == j + 1) {  // wave 0: the next column, rows j+3 .. n-1
          nrm = wave_sum(nrm);
          if (lane == 0) cn[(j + 1) & 1] = nrm;
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    if (n >= 2) {
      dd[n - 2] = A[(n - 2) + (int64_t)(n - 2) * ldA];
      ee[n - 2] = A[(n - 1) + (int64_t)(n - 2) * ldA];
      tau[n - 2] = 0.0;
    }
    dd[n - 1] = A[(n - 1) + (int64_t)(n - 1) * ldA];
    ee[n - 1] = 0.0;
  }
  __syncthreads();

  SYEV_MARK(1);
  // ---- 2. eigenvalues by multisection -------------------------------------
  // Counts run on T scaled by a power of two (exact) to norm in [1, 2);
  // each group of g lanes probes K g points of its eigenvalue's interval.
  double* D = sv;    // diagonal, unscaled (eigenvector phase)
  double* E2 = sw;   // squared off-diagonal, scaled
  double* Ds = Gc;   // diagonal, scaled (Gc is free until the cluster phase)
  double lo_g = 1e308, hi_g = -1e308;
  for (int i = tid; i < n; i += NT) {
    D[i] = dd[i];
    const double el = (i > 0) ? fabs(ee[i - 1]) : 0.0;
    const double er = (i < n - 1) ? fabs(ee[i]) : 0.0;
    lo_g = fmin(lo_g, dd[i] - el - er);
    hi_g = fmax(hi_g, dd[i] + el + er);
  }
  lo_g = blk_min<NT>(lo_g, red);
  hi_g = blk_max<NT>(hi_g, red);
  double tnorm = fmax(fabs(lo_g), fabs(hi_g));
  const bool zero_mat = !(tnorm > 0.0);
  if (zero_mat) tnorm = 1.0;
  const int ex = ilogb(tnorm);
  const double sc = ldexp(1.0, -ex), usc = ldexp(1.0, ex);
  for (int i = tid; i < n; i += NT) {
    Ds[i] = dd[i] * sc;
    if (i < n - 1) {
      const double es = ee[i] * sc;
      E2[i] = es * es;
    }
  }
  __syncthreads();
  const double tn_s = tnorm * sc;
  const double fudge = 4.0 * eps * tn_s;
  const double atol = 0.5 * eps * tn_s;
  const double lo0 = lo_g * sc - fudge, hi0 = hi_g * sc + fudge;
  // only the nv wanted (largest) eigenvalues are located; K points per lane
  // (1 when the groups fill at least half the workgroup, else 2 or 4: the
  // recurrences of one lane are independent, so they overlap)
  int g = 1;
  while (g < 64 && 2 * g * nv <= NT) g *= 2;  // g lanes per wanted eigenvalue
  const int groups = NT / g;
  const int gl = tid % g, gi = tid / g;
  const int busy = g * (nv < groups ? nv : groups);
  auto locate = [&](auto kc) {
    constexpr int K = decltype(kc)::value;
    const double inv_p = 1.0 / (double)(K * g + 1);
    for (int base = n - nv; base < n; base += groups) {
      const int i = base + gi;
      if (i >= n) continue;
      double lo = lo0, hi = hi0;
      for (int it = 0; it < 200; ++it) {
        if (hi - lo <= fmax(atol, 2.0 * eps * fmax(fabs(lo), fabs(hi)))) break;
        const double step = (hi - lo) * inv_p;
        double x[K];
        int cnt[K];
#pragma unroll
        for (int q = 0; q < K; ++q) x[q] = lo + (double)(gl * K + q + 1) * step;
        sturm_counts<K>(n, Ds, E2, x, cnt);
        double nlo = lo, nhi = hi;
#pragma unroll
        for (int q = 0; q < K; ++q) {
          if (cnt[q] <= i) nlo = fmax(nlo, x[q]);
          if (cnt[q] > i) nhi = fmin(nhi, x[q]);
        }
        // the g lanes of a group are aligned to g, so the exchanges stay inside it
        if (g >= 2) {
          nlo = fmax(nlo, dpp_f64<kDppXor1>(nlo));
          nhi = fmin(nhi, dpp_f64<kDppXor1>(nhi));
        }
        if (g >= 4) {
          nlo = fmax(nlo, dpp_f64<kDppXor2>(nlo));
          nhi = fmin(nhi, dpp_f64<kDppXor2>(nhi));
        }
        if (g >= 8) {
          nlo = fmax(nlo, dpp_f64<kDppMirror8>(nlo));
          nhi = fmin(nhi, dpp_f64<kDppMirror8>(nhi));
        }
        if (g >= 16) {
          nlo = fmax(nlo, dpp_f64<kDppMirror16>(nlo));
          nhi = fmin(nhi, dpp_f64<kDppMirror16>(nhi));
        }
        for (int m = 16; m < g; m <<= 1) {
          nlo = fmax(nlo, __shfl_xor(nlo, m));
          nhi = fmin(nhi, __shfl_xor(nhi, m));
        }
        if (!(nlo < nhi)) break;
        lo = nlo;
        hi = nhi;
      }
      if (gl == 0) lamv[i] = (0.5 * (lo + hi)) * usc;
    }
  };
  if (2 * busy >= NT)
    locate(std::integral_constant<int, 1>{});
  else if (4 * busy >= NT)
    locate(std::integral_constant<int, 2>{});
  else
    locate(std::integral_constant<int, 4>{});
  __syncthreads();

  SYEV_MARK(2);
  // ---- 3. eigenvectors of T by inverse iteration ---------------------------
  const int n0 = n - nv;  // first computed eigenvalue index
  const double tiny = eps * tnorm;
  // clusters: consecutive gaps within ctol ||T|| (the caller's, else 1e-8;
  // in the default mode a whole-block correction follows, which needs the
  // vectors of separate clusters to overlap by no more than about 1e-8)
  const bool correct_all = !(ctol_rel > 0.0);
  const double ctol = (ctol_rel > 0.0 ? ctol_rel : 1e-8) * tnorm;
  // the off-diagonal into LDS (Gc is free between the eigenvalue and the
  // cluster phases), so the factorisation's loop reads no global memory
  double* EL = Gc;
  for (int i = tid; i < n - 1; i += NT) EL[i] = ee[i];
  __syncthreads();
  // The eigenvectors of T (Zt) live in LDS past the working matrix when the
  // launch reserved room for them, else in the work area; the two phases
  // below are instantiated for each, so that LDS accesses compile to LDS
  // instructions.
  auto vectors_of_t = [&](double* __restrict__ Zt) __attribute__((always_inline)) {
  for (int slot0 = 0; slot0 < nv; slot0 += NT) {
    const int slot = slot0 + tid;
    if (slot < nv) {
      const int i = n0 + slot;
      double* lu = lub + tid;
      tri_factor<NT>(n, D, EL, lamv[i], tiny, lu, nmax);
      double* y = Zt + slot;
      random_start(n, i, y, nv);
      // two solves from a random start: with lambda accurate to a few ulps of
      // ||T|| the first leaves components outside the eigenvalue's cluster of
      // relative size eps ||T|| / gap, the second squares that
      for (int it = 0; it < 2; ++it) {
        tri_solve<NT>(n, lu, nmax, y, nv);
        normalize_serial(n, y, nv);
      }
    }
  }
  __syncthreads();

  SYEV_MARK(3);
  // largest cluster orthonormalised by Cholesky QR (its Gram matrix in Gc)
  int cmax = kClusterMax;
  if (lds_a) {
    const int64_t gcap = syev_lds_gc(nmax);
    while ((int64_t)cmax * cmax > gcap) --cmax;
  }
  // ---- 3b. orthonormalise clusters of close eigenvalues --------------------
  // The independent iterates of a cluster (gap <= ctol) span its invariant
  // subspace; they are orthonormalised together, which mixes only vectors of
  // eigenvalues closer than ctol.
  {
    int a = n0;
    while (a < n) {
      int b = a + 1;
      while (b < n && (lamv[b] - lamv[b - 1]) <= ctol) ++b;
      const int c = b - a;
      if (c > 1 && c <= cmax) {
        const int s0 = a - n0;
        for (int pass = 0; pass < 2; ++pass) {
          const int np = c * (c + 1) / 2;
          for (int p = tid; p < np; p += NT) {
            int i = 0;
            while ((i + 1) * (i + 2) / 2 <= p) ++i;
            const int jj = p - i * (i + 1) / 2;
            Gc[i + jj * c] = dot_pipe<DU>(Zt + s0 + i, nv, Zt + s0 + jj, nv, n);
          }
          __syncthreads();
          for (int jc = 0; jc < c; ++jc) {  // Cholesky G = L L^T, lower triangle
            if (tid == 0) Gc[jc + jc * c] = sqrt(fmax(Gc[jc + jc * c], 1e-300));
            __syncthreads();
            for (int i = jc + 1 + tid; i < c; i += NT) Gc[i + jc * c] /= Gc[jc + jc * c];
            __syncthreads();
            const int rem = c - jc - 1;
            for (int e = tid; e < rem * rem; e += NT) {
              const int cc = jc + 1 + e / rem, r = jc + 1 + e % rem;
              if (r >= cc) Gc[r + cc * c] -= Gc[r + jc * c] * Gc[cc + jc * c];
            }
            __syncthreads();
          }
          // each row z of the cluster block becomes z L^{-T} (forward substitution)
          for (int pos = tid; pos < n; pos += NT) {
            double* zr = Zt + (int64_t)pos * nv + s0;
            for (int j2 = 0; j2 < c; ++j2) {
              double sacc = zr[j2];
              for (int i = 0; i < j2; ++i) sacc -= zr[i] * Gc[j2 + i * c];
              zr[j2] = sacc / Gc[j2 + j2 * c];
            }
          }
          __syncthreads();
        }
      } else if (c > cmax) {
        // classical Gram-Schmidt run twice, vector by vector, by the whole
        // workgroup: wave w forms the coefficients against vectors w, w+NW,
        // ... of the cluster (Gc), then every thread updates its positions
        const int s0 = a - n0;
        for (int i = 0; i < c; ++i) {
          double* y = Zt + s0 + i;
          for (int pass = 0; pass < 2 && i > 0; ++pass) {
            for (int q = wid; q < i; q += NW) {
              const double* zq = Zt + s0 + q;
              double dot = 0.0;
              for (int pos = lane; pos < n; pos += 64)
                dot += zq[(int64_t)pos * nv] * y[(int64_t)pos * nv];
              dot = wave_sum(dot);
              if (lane == 0) Gc[q] = dot;
            }
            __syncthreads();
            for (int pos = tid; pos < n; pos += NT) {
              const double* zr = Zt + (int64_t)pos * nv + s0;
              double acc = 0.0;
              for (int q = 0; q < i; ++q) acc += Gc[q] * zr[q];
              y[(int64_t)pos * nv] -= acc;
            }
            __syncthreads();
          }
          double ss = 0.0;
          for (int pos = tid; pos < n; pos += NT) ss += y[(int64_t)pos * nv] * y[(int64_t)pos * nv];
          ss = blk_sum<NT>(ss, red);
          const double sc = (ss > 0.0) ? 1.0 / sqrt(ss) : 0.0;
          for (int pos = tid; pos < n; pos += NT) y[(int64_t)pos * nv] *= sc;
          __syncthreads();
        }
      }
      a = b;
    }
  }
  __syncthreads();
  // the LU arrays are free once every vector has been iterated
  if (correct_all && nv > 1) wg_orth_correct<NT>(n, nv, Zt, lub, lub + (int64_t)nv * nv, red);
  };
  if (zt_lds)
    vectors_of_t(ZtL);
  else
    vectors_of_t(ZtG);
  double* const Zt = zt_lds ? ZtL : ZtG;

  SYEV_MARK(4);
  if (NT <= 512 && lds_a) {
    // ---- 4/5. Z = H_0 (H_1 ( ... (H_{n-3} Z_T))) --------------------------
    // Each wanted vector is owned by 8 lanes, lane k holding positions
    // k, k+8, ... in registers; a reflector costs those lanes one dot
    // product (summed by three butterflies) and one axpy, with v read from
    // LDS, so no barrier is needed.
    constexpr int PL = (kLdsMax + 7) / 8;
    const double* const AL = smem;
    for (int i = tid; i < n; i += NT) sv[i] = (i < n - 2) ? tau[i] : 0.0;
    for (int i = tid; i < n; i += NT) wq[i] = (zero_mat || i < n - nv) ? 0.0 : lamv[i];
    __syncthreads();
    const int k8 = tid & 7;
    for (int slot0 = 0; slot0 < nv; slot0 += NT / 8) {
      const int slot = slot0 + (tid >> 3);
      const bool act = slot < nv;
      double z[PL];
#pragma unroll
      for (int i = 0; i < PL; ++i) {
        const int pos = k8 + 8 * i;
        z[i] = (act && pos < n) ? Zt[(int64_t)pos * nv + slot] : 0.0;
      }
      // reflector j-1 is loaded while reflector j is applied
      double vv[PL], tj = 0.0;
#pragma unroll
      for (int i = 0; i < PL; ++i) vv[i] = 0.0;
      if (n >= 3) {
        const double* v = AL + (int64_t)(n - 3) * ldA;
        tj = sv[n - 3];
#pragma unroll
        for (int i = 0; i < PL; ++i) {
          const int pos = k8 + 8 * i;
          vv[i] = (pos >= n - 1 && pos < n) ? v[pos] : (pos == n - 2 ? 1.0 : 0.0);
        }
      }
      for (int j = n - 3; j >= 0; --j) {
        double vn[PL], tn = 0.0;
        const int jn = j > 0 ? j - 1 : 0;
        const double* v = AL + (int64_t)jn * ldA;
#pragma unroll
        for (int i = 0; i < PL; ++i) {
          const int pos = k8 + 8 * i;
          vn[i] = (pos >= jn + 2 && pos < n) ? v[pos] : (pos == jn + 1 ? 1.0 : 0.0);
        }
        tn = sv[jn];
        if (tj != 0.0) {
          double part = 0.0;
#pragma unroll
          for (int i = 0; i < PL; ++i) part += vv[i] * z[i];
          part += dpp_f64<kDppXor1>(part);
          part += dpp_f64<kDppXor2>(part);
          part += dpp_f64<kDppMirror8>(part);
          const double f = tj * part;
#pragma unroll
          for (int i = 0; i < PL; ++i) z[i] -= f * vv[i];
        }
#pragma unroll
        for (int i = 0; i < PL; ++i) vv[i] = vn[i];
        tj = tn;
      }
      if (act) {
#pragma unroll
        for (int i = 0; i < PL; ++i) {
          const int pos = k8 + 8 * i;
          if (pos < n) Zq[pos + (int64_t)(n0 + slot) * ldz] = z[i];
        }
      }
    }
    SYEV_MARK(5);
    SYEV_MARK(6);
    return;
  }
  {
    // ---- 4/5 (global path). Z = H_0 (H_1 ( ... (H_{n-3} Z_T))) on panels of
    // the wanted vectors held in LDS, with blocks of RB reflectors staged in
    // LDS (one barrier per block).  A vector is owned by g lanes of one wave
    // (lane k: positions k, k+g, ...), so applying a reflector needs only an
    // in-wave reduction and an in-order LDS update.
    const int64_t stage_d = kLdsDoubles - 2 * nmax - 32;
    const int RB = (int)std::min<int64_t>(16, std::max<int64_t>(1, stage_d / (4 * (int64_t)n)));
    double* vb = stage;             // RB x n
    double* zp = stage + RB * n;    // nvp x n
    const int nvp = (int)std::min<int64_t>(nv, (stage_d - RB * (int64_t)n) / n);
    for (int i = tid; i < n; i += NT) wq[i] = (zero_mat || i < n - nv) ? 0.0 : lamv[i];
    for (int slot0 = 0; slot0 < nv; slot0 += nvp) {
      const int cnt = std::min(nvp, nv - slot0);
      for (int e = tid; e < cnt * n; e += NT) {
        const int sl = e / n, pos = e - sl * n;
        zp[e] = Zt[(int64_t)pos * nv + slot0 + sl];
      }
      int g = 64;
      while (g > 1 && g * cnt > NT) g >>= 1;
      const int sl = tid / g, k = tid % g;
      for (int jb = n - 3; jb >= 0; jb -= RB) {
        const int j0 = jb - RB + 1 > 0 ? jb - RB + 1 : 0;
        __syncthreads();  // the previous block is no longer read
        for (int e = tid; e < (jb - j0 + 1) * n; e += NT) {
          const int q = e / n, pos = e - q * n, j = j0 + q;
          vb[e] = (pos < j + 1) ? 0.0 : (pos == j + 1 ? 1.0 : gA[pos + (int64_t)j * ldA]);
        }
        __syncthreads();
        if (sl < cnt) {
          double* z = zp + (int64_t)sl * n;
          for (int j = jb; j >= j0; --j) {
            const double tj = tau[j];
            if (tj == 0.0) continue;
            const double* v = vb + (int64_t)(j - j0) * n;
            double part = 0.0;
            for (int pos = j + 1 + k; pos < n; pos += g) part += v[pos] * z[pos];
            if (g >= 2) part += dpp_f64<kDppXor1>(part);
            if (g >= 4) part += dpp_f64<kDppXor2>(part);
            if (g >= 8) part += dpp_f64<kDppMirror8>(part);
            if (g >= 16) part += dpp_f64<kDppMirror16>(part);
            if (g >= 32) part += __shfl_xor(part, 16);
            if (g >= 64) part += __shfl_xor(part, 32);
            const double f = tj * part;
            for (int pos = j + 1 + k; pos < n; pos += g) z[pos] -= f * v[pos];
            __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
          }
        }
      }
      __syncthreads();
      for (int e = tid; e < cnt * n; e += NT) {
        const int s2 = e / n, pos = e - s2 * n;
        Zq[pos + (int64_t)(n0 + slot0 + s2) * ldz] = zp[e];
      }
      __syncthreads();
    }
    SYEV_MARK(5);
    SYEV_MARK(6);
    return;
  }
}

bool syev_timing = false;

template <int NT>
hipError_t syev_launch_t(const SyevArgs* sarr, int64_t batch, int64_t n, const int* ns,
                         const double* A, int64_t lda, int64_t strideA, double* w, int64_t stridew,
                         double* Z, int64_t ldz, int64_t strideZ, int64_t nvec, double* work,
                         hipStream_t s, double ctol, int64_t nvmax) {
  const bool lds_a = n <= kLdsMax && NT <= 512;
  const int64_t lds_cap = syev_lds_alloc(n, nvmax, lds_a);
  const size_t lds = (size_t)lds_cap * sizeof(double);
  static bool attr_set = false;
  if (!attr_set) {
    hipError_t e = hipFuncSetAttribute((const void*)syev_kernel<NT>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e != hipSuccess) return e;
    attr_set = true;
  }
  hipLaunchKernelGGL(syev_kernel<NT>, dim3((unsigned)batch), dim3(NT), lds, s, sarr, (int)n, ns, A,
                     lda, strideA, w, stridew, Z, ldz, strideZ, (int)nvec, work, n, lds_a ? 1 : 0,
                     syev_timing ? 1 : 0, ctol, lds_cap);
  return hipGetLastError();
}

}  // namespace

void syev_timing_enable(bool on) { syev_timing = on; }

void syev_timing_report(FILE* f) {
  unsigned long long c[8] = {0};
  if (hipMemcpyFromSymbol(c, HIP_SYMBOL(g_syev_cycles), sizeof(c)) != hipSuccess) return;
  const char* names[7] = {"copy", "tridiag", "eigvals", "invit", "clusters", "backtrans", "output"};
  std::fprintf(f, "[eda] syev cycles (matrix 0 of every launch):");
  for (int i = 0; i < 7; ++i) std::fprintf(f, " %s=%llu", names[i], c[i]);
  std::fprintf(f, "\n");
}

size_t syev_work_bytes(int64_t nmax) {
  // the larger thread count sizes the per-thread LU storage
  return (size_t)syev_work_doubles(nmax, 1024) * sizeof(double);
}

hipError_t launch_syev(int64_t batch, int64_t n, const int* ns, const double* A, int64_t lda,
                       int64_t strideA, double* w, int64_t stridew, double* Z, int64_t ldz,
                       int64_t strideZ, int64_t nvec, double* work, hipStream_t s, double ctol) {
  if (n < 1 || n > SYEV_NMAX || batch < 1) return hipErrorInvalidValue;
  // workgroup size by measurement: 256 threads up to n = 48, 512 while the
  // matrix fits in LDS, 1024 for the global-memory path
  const int64_t nvmax = (nvec <= 0 || nvec > n) ? n : nvec;
  if (n <= 48)
    return syev_launch_t<256>(nullptr, batch, n, ns, A, lda, strideA, w, stridew, Z, ldz, strideZ,
                              nvec, work, s, ctol, nvmax);
  if (n <= kLdsMax)
    return syev_launch_t<512>(nullptr, batch, n, ns, A, lda, strideA, w, stridew, Z, ldz, strideZ,
                              nvec, work, s, ctol, nvmax);
  return syev_launch_t<1024>(nullptr, batch, n, ns, A, lda, strideA, w, stridew, Z, ldz, strideZ,
                             nvec, work, s, ctol, nvmax);
}

// Several problems of different size: `dev` holds the count entries on the
// device; every entry's work area must hold syev_work_bytes(max n).
hipError_t launch_syev_multi(int count, const SyevArgs* host, const SyevArgs* dev,
                             hipStream_t s) {
  if (count < 1) return hipSuccess;
  int64_t nmax = 0, nvmax = 0;
  for (int p = 0; p < count; ++p) {
    if (host[p].n < 0 || host[p].n > SYEV_NMAX) return hipErrorInvalidValue;
    nmax = std::max(nmax, host[p].n);
    const int64_t nv = (host[p].nvec <= 0 || host[p].nvec > host[p].n) ? host[p].n : host[p].nvec;
    nvmax = std::max(nvmax, nv);
  }
  if (nmax == 0) return hipSuccess;
  if (count == 1) {
    const SyevArgs& a = host[0];
    return launch_syev(1, a.n, nullptr, a.A, a.lda, 0, a.w, 0, a.Z, a.ldz, 0, a.nvec, a.work, s,
                       a.ctol);
  }
  if (nmax <= 48)
    return syev_launch_t<256>(dev, count, nmax, nullptr, nullptr, 0, 0, nullptr, 0, nullptr, 0, 0,
                              0, nullptr, s, 0.0, nvmax);
  if (nmax <= kLdsMax)
    return syev_launch_t<512>(dev, count, nmax, nullptr, nullptr, 0, 0, nullptr, 0, nullptr, 0, 0,
                              0, nullptr, s, 0.0, nvmax);
  return syev_launch_t<1024>(dev, count, nmax, nullptr, nullptr, 0, 0, nullptr, 0, nullptr, 0, 0,
                             0, nullptr, s, 0.0, nvmax);
}

}  // namespace eda
