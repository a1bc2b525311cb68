// Dense symmetric eigensolver for the small matrices of the method: the
// Gram blocks H_W^T H_W and H_B^T H_B (whose eigenpairs give the cores
// V phi(Lambda) V^T of the exponentials) and the Rayleigh-Ritz matrices of
// block Lanczos.  One 1024-thread workgroup per matrix (batched over the
// grid), float64 throughout.
//
//   1. Householder reduction to tridiagonal form T = Q^T A Q (unblocked:
//      per column one reflector, one symmetric matrix-vector product, one
//      rank-2 update; the working copy of A stays in L2).
//   2. Eigenvalues of T by Sturm-count bisection; the workgroup's threads
//      are split into groups of g lanes that probe g points per step
//      (multisection), so small matrices converge in few steps.
//   3. Eigenvectors of T by inverse iteration, one thread per eigenvalue
//      (LU with partial pivoting of T - lambda I, three solves), then
//      modified Gram-Schmidt inside clusters of close eigenvalues.
//   4. Back-transformation by the stored reflectors, one thread per vector.
#include "common.h"

namespace eda {

namespace {

constexpr int ST = 1024;      // threads per workgroup
constexpr int NW = ST / 64;   // waves
constexpr int SYEV_NMAX = 2048;

__device__ __forceinline__ double wave_sum(double v) {
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  return v;
}

__device__ __forceinline__ double blk_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < NW; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double blk_max(double v, double* red) {
  for (int m = 32; m >= 1; m >>= 1) v = fmax(v, __shfl_xor(v, m));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < NW; ++w) s = fmax(s, red[w]);
  return s;
}

__device__ __forceinline__ double blk_min(double v, double* red) {
  for (int m = 32; m >= 1; m >>= 1) v = fmin(v, __shfl_xor(v, m));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = red[0];
  for (int w = 1; w < NW; ++w) s = fmin(s, red[w]);
  return s;
}

__device__ __forceinline__ uint64_t hash64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}

// Number of eigenvalues of T below x (Sturm count of the LDL^T pivots).
__device__ __forceinline__ int sturm_count(int n, const double* __restrict__ D,
                                           const double* __restrict__ E2, double x,
                                           double pivmin) {
  double q = D[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  int c = (q < 0.0);
  for (int k = 1; k < n; ++k) {
    q = (D[k] - x) - E2[k - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += (q < 0.0);
  }
  return c;
}

// LU factorisation with partial pivoting of T - lam I (T tridiagonal: diagonal
// D, off-diagonal ee).  Stored per position k with stride ST: 1/U(k,k),
// U(k,k+1), U(k,k+2), the multiplier and the interchange flag.
__device__ void tri_factor(int n, const double* __restrict__ D, const double* __restrict__ ee,
                           double lam, double tiny, double* __restrict__ lu, int64_t nmax) {
  double* U1 = lu;
  double* U2 = lu + nmax * ST;
  double* U3 = lu + 2 * nmax * ST;
  double* Lm = lu + 3 * nmax * ST;
  double* Pv = lu + 4 * nmax * ST;
#define LU(arr, k) arr[(int64_t)(k) * ST]
  double p = D[0] - lam;
  double qv = (n > 1) ? ee[0] : 0.0;
  double rv = 0.0;
  for (int k = 0; k < n - 1; ++k) {
    const double ek = ee[k];
    const double an = D[k + 1] - lam;
    const double en = (k + 1 < n - 1) ? ee[k + 1] : 0.0;
    if (fabs(p) >= fabs(ek)) {
      if (fabs(p) < tiny) p = (p < 0.0) ? -tiny : tiny;
      const double l = ek / p;
      LU(U1, k) = 1.0 / p;
      LU(U2, k) = qv;
      LU(U3, k) = rv;
      LU(Lm, k) = l;
      LU(Pv, k) = 0.0;
      p = an - l * qv;
      qv = en - l * rv;
    } else {
      const double l = p / ek;
      LU(U1, k) = 1.0 / ek;
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
// rescales the computed tail whenever it grows past 2^300, so chains of tiny
// pivots (split matrices, multiple eigenvalues) cannot overflow.
__device__ void tri_solve(int n, const double* __restrict__ lu, int64_t nmax,
                          double* __restrict__ y, int64_t ys) {
  const double* U1 = lu;
  const double* U2 = lu + nmax * ST;
  const double* U3 = lu + 2 * nmax * ST;
  const double* Lm = lu + 3 * nmax * ST;
  const double* Pv = lu + 4 * nmax * ST;
#define LU(arr, k) arr[(int64_t)(k) * ST]
#define YV(k) y[(int64_t)(k) * ys]
  // forward elimination; the running entry stays in a register
  double carry = YV(0);
  for (int k = 0; k < n - 1; ++k) {
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
  for (int k = n - 1; k >= 0; --k) {
    double x = (YV(k) - LU(U2, k) * x1 - LU(U3, k) * x2) * LU(U1, k);
    if (!(fabs(x) < big)) {
      // rescale the whole system (right-hand side of rows < k and the
      // solution of rows > k) so the remaining steps stay finite
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

__device__ void random_start(int n, int i, double* y, int64_t ys, int first, int step) {
  for (int k = first; k < n; k += step) {
    const uint64_t h = hash64(((uint64_t)(i + 1) << 32) ^ (uint64_t)k ^ 0x5bd1e995ull);
    y[(int64_t)k * ys] = ((double)(h >> 11) * 0x1.0p-53) * 2.0 - 1.0;
  }
}

__device__ void normalize_serial(int n, double* y, int64_t ys) {
  double mx = 0.0;
  for (int k = 0; k < n; ++k) mx = fmax(mx, fabs(y[(int64_t)k * ys]));
  const double inv = (mx > 0.0) ? 1.0 / mx : 1.0;
  double nrm = 0.0;
  for (int k = 0; k < n; ++k) {
    const double v = y[(int64_t)k * ys] * inv;
    nrm += v * v;
  }
  const double sc = inv / sqrt(nrm);
  for (int k = 0; k < n; ++k) y[(int64_t)k * ys] *= sc;
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

struct SyevWork {
  double* A;    // n x n working copy (ld n), later the reflectors
  double* dd;   // diagonal of T
  double* ee;   // off-diagonal of T
  double* tau;  // reflector scalars
  double* lam;  // eigenvalues ascending
  double* Zt;   // eigenvectors of T, layout [pos][slot] (n x nv)
  double* lu;   // LU of T - lambda I, layout [array][pos][thread]
};

__device__ SyevWork carve(double* base, int64_t nmax) {
  SyevWork w;
  w.A = base;
  w.dd = w.A + nmax * nmax;
  w.ee = w.dd + nmax;
  w.tau = w.ee + nmax;
  w.lam = w.tau + nmax;
  w.Zt = w.lam + nmax;
  w.lu = w.Zt + nmax * nmax;
  return w;
}

__global__ __launch_bounds__(ST) void syev_kernel(int nfix, const int* __restrict__ ns,
                                                  const double* __restrict__ Ain, int64_t lda,
                                                  int64_t strideA, double* __restrict__ wout,
                                                  int64_t stridew, double* __restrict__ Zout,
                                                  int64_t ldz, int64_t strideZ, int nvec_req,
                                                  double* __restrict__ work, int64_t nmax) {
  __shared__ double sbuf[2 * SYEV_NMAX];
  __shared__ double red[NW];
  double* sv = sbuf;
  double* sw = sbuf + SYEV_NMAX;
  const int q = blockIdx.x;
  const int n = (ns != nullptr) ? ns[q] : nfix;
  if (n <= 0) return;
  const int nv = (nvec_req <= 0 || nvec_req > n) ? n : nvec_req;
  const double* Aq = Ain + q * strideA;
  double* wq = wout + q * stridew;
  double* Zq = Zout + q * strideZ;
  const int64_t wstride = 5 * nmax + 2 * nmax * nmax + 5 * nmax * (int64_t)ST;
  SyevWork W = carve(work + q * wstride, nmax);
  double* A = W.A;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const double eps = 0x1.0p-53;

  // ---- 0. symmetrised working copy (lower triangle of the input) ---------
  for (int64_t e = tid; e < (int64_t)n * n; e += ST) {
    const int c = (int)(e / n), r = (int)(e - (int64_t)c * n);
    A[r + (int64_t)c * n] = (r >= c) ? Aq[r + c * lda] : Aq[c + r * lda];
  }
  __syncthreads();

  // ---- 1. Householder tridiagonalisation ---------------------------------
  for (int j = 0; j < n - 2; ++j) {
    const int m1 = n - j - 1;
    double* col = A + (int64_t)j * n;
    double s = 0.0;
    for (int r = j + 2 + tid; r < n; r += ST) s += col[r] * col[r];
    s = blk_sum(s, red);
    const double alpha = col[j + 1];
    double beta, tau, scale;
    if (s == 0.0) {
      tau = 0.0;
      beta = alpha;
      scale = 0.0;
    } else {
      beta = -copysign(sqrt(alpha * alpha + s), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    for (int r = j + 1 + tid; r < n; r += ST) sv[r] = (r == j + 1) ? 1.0 : col[r] * scale;
    __syncthreads();
    for (int r = j + 2 + tid; r < n; r += ST) col[r] = sv[r];
    if (tid == 0) {
      W.dd[j] = A[j + (int64_t)j * n];
      W.ee[j] = beta;
      W.tau[j] = tau;
    }
    if (tau == 0.0) {
      __syncthreads();
      continue;
    }
    // p = tau * A22 v, one wave per column (A22 symmetric, columns contiguous)
    for (int r = j + 1 + wid; r < n; r += NW) {
      const double* ac = A + (int64_t)r * n;
      double acc = 0.0;
      for (int c = j + 1 + lane; c < n; c += 64) acc += ac[c] * sv[c];
      acc = wave_sum(acc);
      if (lane == 0) sw[r] = tau * acc;
    }
    __syncthreads();
    double kk = 0.0;
    for (int r = j + 1 + tid; r < n; r += ST) kk += sw[r] * sv[r];
    kk = blk_sum(kk, red);
    const double K = 0.5 * tau * kk;
    for (int r = j + 1 + tid; r < n; r += ST) sw[r] -= K * sv[r];
    __syncthreads();
    const int64_t mm = (int64_t)m1 * m1;
    for (int64_t e = tid; e < mm; e += ST) {
      const int c = j + 1 + (int)(e / m1), r = j + 1 + (int)(e % m1);
      A[r + (int64_t)c * n] -= sv[r] * sw[c] + sw[r] * sv[c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      W.dd[n - 2] = A[(n - 2) + (int64_t)(n - 2) * n];
      W.ee[n - 2] = A[(n - 1) + (int64_t)(n - 2) * n];
      W.tau[n - 2] = 0.0;
    }
    W.dd[n - 1] = A[(n - 1) + (int64_t)(n - 1) * n];
    W.ee[n - 1] = 0.0;
  }
  __syncthreads();

  // ---- 2. eigenvalues by multisection -------------------------------------
  double* D = sv;
  double* E2 = sw;
  double lo_g = 1e308, hi_g = -1e308, e2max = 0.0;
  for (int i = tid; i < n; i += ST) {
    D[i] = W.dd[i];
    const double el = (i > 0) ? fabs(W.ee[i - 1]) : 0.0;
    const double er = (i < n - 1) ? fabs(W.ee[i]) : 0.0;
    if (i < n - 1) {
      E2[i] = W.ee[i] * W.ee[i];
      e2max = fmax(e2max, E2[i]);
    }
    lo_g = fmin(lo_g, W.dd[i] - el - er);
    hi_g = fmax(hi_g, W.dd[i] + el + er);
  }
  lo_g = blk_min(lo_g, red);
  hi_g = blk_max(hi_g, red);
  e2max = blk_max(e2max, red);
  double tnorm = fmax(fabs(lo_g), fabs(hi_g));
  const bool zero_mat = !(tnorm > 0.0);
  if (zero_mat) tnorm = 1.0;
  const double pivmin = 2.2250738585072014e-308 * fmax(1.0, e2max);
  const double fudge = 2.0 * eps * tnorm + 2.0 * pivmin;
  const double atol = 0.5 * eps * tnorm;
  int g = 1;
  while (g < 64 && 2 * g * n <= ST) g *= 2;
  const int groups = ST / g;
  const int gl = tid % g, gi = tid / g;
  for (int base = 0; base < n; base += groups) {
    const int i = base + gi;
    if (i < n) {
      double lo = lo_g - fudge, hi = hi_g + fudge;
      for (int it = 0; it < 200; ++it) {
        if (hi - lo <= fmax(atol, 2.0 * eps * fmax(fabs(lo), fabs(hi)))) break;
        const double x = lo + (double)(gl + 1) * ((hi - lo) / (double)(g + 1));
        const int cnt = sturm_count(n, D, E2, x, pivmin);
        double nlo = (cnt <= i) ? x : lo;
        double nhi = (cnt > i) ? x : hi;
        for (int m = 1; m < g; m <<= 1) {
          nlo = fmax(nlo, __shfl_xor(nlo, m));
          nhi = fmin(nhi, __shfl_xor(nhi, m));
        }
        if (!(nlo < nhi)) break;
        lo = nlo;
        hi = nhi;
      }
      if (gl == 0) W.lam[i] = 0.5 * (lo + hi);
    }
  }
  __syncthreads();

  // ---- 3. eigenvectors of T by inverse iteration ---------------------------
  // Every wanted eigenvector is computed independently, one thread each
  // (random start, three solves with T - lambda I).  Eigenvalues closer than
  // ctol (relative to ||T||) form a cluster, whose vectors are then
  // orthonormalised together by modified Gram-Schmidt (twice), one wave per
  // cluster: the independent iterates span the cluster's invariant subspace,
  // and within it mixing only happens between eigenvalues closer than ctol.
  const int n0 = n - nv;  // first computed eigenvalue index
  const double tiny = eps * tnorm;
  const double ctol = 1e-3 * tnorm;
  for (int slot0 = 0; slot0 < nv; slot0 += ST) {
    const int slot = slot0 + tid;
    if (slot < nv) {
      const int i = n0 + slot;
      double* lu = W.lu + tid;
      tri_factor(n, D, W.ee, W.lam[i], tiny, lu, nmax);
      double* y = W.Zt + slot;
      random_start(n, i, y, nv, 0, 1);
      for (int it = 0; it < 3; ++it) {
        tri_solve(n, lu, nmax, y, nv);
        normalize_serial(n, y, nv);
      }
    }
  }
  __syncthreads();
  {
    int cl = 0;
    int a = n0;
    while (a < n) {
      int b = a + 1;
      while (b < n && (W.lam[b] - W.lam[b - 1]) <= ctol) ++b;
      if (b - a > 1) {
        if ((cl % NW) == wid) {
          for (int pass = 0; pass < 2; ++pass) {
            for (int i = a; i < b; ++i) {
              double* y = W.Zt + (i - n0);
              for (int k = a; k < i; ++k) {
                const double* zk = W.Zt + (k - n0);
                double dot = 0.0;
                for (int pos = lane; pos < n; pos += 64)
                  dot += zk[(int64_t)pos * nv] * y[(int64_t)pos * nv];
                dot = wave_sum(dot);
                for (int pos = lane; pos < n; pos += 64) y[(int64_t)pos * nv] -= dot * zk[(int64_t)pos * nv];
              }
              wave_normalize(n, y, nv, lane);
              __threadfence_block();
            }
          }
        }
        ++cl;
      }
      a = b;
    }
  }
  __syncthreads();

  // ---- 4. back-transformation z <- H_0 H_1 ... H_{n-3} z ------------------
  {
    const int rb = (n > 0) ? (int)std::max<int64_t>(1, (int64_t)(2 * SYEV_NMAX) / n) : 1;
    double* R = sbuf;  // reflectors staged in LDS: rb x n <= 2 * SYEV_NMAX
    for (int jt = n - 3; jt >= 0; jt -= rb) {
      const int jb = std::max(0, jt - rb + 1);  // reflectors jb..jt
      __syncthreads();
      for (int64_t e = tid; e < (int64_t)(jt - jb + 1) * n; e += ST) {
        const int jj = (int)(e / n), r = (int)(e - (int64_t)jj * n);
        const int j = jb + jj;
        double v = 0.0;
        if (r == j + 1) v = 1.0;
        else if (r > j + 1) v = A[r + (int64_t)j * n];
        R[e] = v;
      }
      __syncthreads();
      for (int slot = tid; slot < nv; slot += ST) {
        double* z = W.Zt + slot;
        for (int j = jt; j >= jb; --j) {
          const double tj = W.tau[j];
          if (tj == 0.0) continue;
          const double* v = R + (int64_t)(j - jb) * n;
          double s = 0.0;
          for (int r = j + 1; r < n; ++r) s += v[r] * z[(int64_t)r * nv];
          s *= tj;
          for (int r = j + 1; r < n; ++r) z[(int64_t)r * nv] -= s * v[r];
        }
      }
    }
  }
  __syncthreads();

  // ---- 5. outputs ----------------------------------------------------------
  for (int i = tid; i < n; i += ST) wq[i] = zero_mat ? 0.0 : W.lam[i];
  for (int64_t e = tid; e < (int64_t)nv * n; e += ST) {
    const int slot = (int)(e / n), pos = (int)(e - (int64_t)slot * n);
    Zq[pos + (int64_t)(n0 + slot) * ldz] = W.Zt[(int64_t)pos * nv + slot];
  }
}

}  // namespace

size_t syev_work_bytes(int64_t nmax) {
  const int64_t per = 5 * nmax + 2 * nmax * nmax + 5 * nmax * (int64_t)ST;
  return (size_t)per * sizeof(double);
}

hipError_t launch_syev(int64_t batch, int64_t n, const int* ns, const double* A, int64_t lda,
                       int64_t strideA, double* w, int64_t stridew, double* Z, int64_t ldz,
                       int64_t strideZ, int64_t nvec, double* work, hipStream_t s) {
  if (n < 1 || n > SYEV_NMAX || batch < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL(syev_kernel, dim3((unsigned)batch), dim3(ST), 0, s, (int)n, ns, A, lda,
                     strideA, w, stridew, Z, ldz, strideZ, (int)nvec, work, n);
  return hipGetLastError();
}

}  // namespace eda
