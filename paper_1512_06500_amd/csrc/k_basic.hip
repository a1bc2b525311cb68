// Elementwise and small helper kernels of libeda.
#include "common.h"

namespace eda {

namespace {

__device__ __forceinline__ double block_sum(double v, double* red) {
  // Fixed-order reduction: wave butterfly, then wave 0 sums the wave partials in order.
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < nw; ++w) s += red[w];
  return s;
}

// ---------------------------------------------------------------------------
// Scatter factors, Section 1, eqs. (1.1)-(1.2), in two launches.  First one
// workgroup per (256 feature rows, class j): each thread sums its row over
// the class's samples, writes the centred samples to H_W and the class sum
// s_j to H_B (column j).  Then one thread per row: mu = (sum_j s_j) / n (the
// sample-weighted global centroid) and H_B(:, j) = sqrt(n_j) (s_j / n_j - mu).
// ---------------------------------------------------------------------------
// A class of at most CM samples is read once: its entries of the thread's
// row stay in registers (all loads issued before the first use; indices
// past the class read its last sample again, a cache hit, and are unused).
// Larger classes read their samples twice.  Either way s is the sum in
// sample order.
template <int CM>
__device__ __forceinline__ void scatter_class_regs(int64_t i, const double* __restrict__ X,
                                                   int64_t ldx, int64_t c0, int64_t nj,
                                                   double* __restrict__ HW, int64_t ldw,
                                                   double& s) {
  double v[CM];
#pragma unroll
  for (int u = 0; u < CM; ++u) v[u] = X[i + (c0 + (u < nj ? u : nj - 1)) * ldx];
  s = 0.0;
#pragma unroll
  for (int u = 0; u < CM; ++u)
    if (u < nj) s += v[u];
  const double mj = s / (double)nj;
#pragma unroll
  for (int u = 0; u < CM; ++u)
    if (u < nj) HW[i + (c0 + u) * ldw] = v[u] - mj;
}

__global__ __launch_bounds__(256) void scatter_class_kernel(int64_t d, const double* __restrict__ X,
                                                            int64_t ldx,
                                                            const int64_t* __restrict__ offs,
                                                            double* __restrict__ HW, int64_t ldw,
                                                            double* __restrict__ HB, int64_t ldb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t j = blockIdx.y;
  if (i >= d) return;
  const int64_t c0 = offs[j], c1 = offs[j + 1], nj = c1 - c0;
  double s = 0.0;
  if (nj <= 8) {
    scatter_class_regs<8>(i, X, ldx, c0, nj, HW, ldw, s);
  } else if (nj <= 16) {
    scatter_class_regs<16>(i, X, ldx, c0, nj, HW, ldw, s);
  } else if (nj <= 24) {
    scatter_class_regs<24>(i, X, ldx, c0, nj, HW, ldw, s);
  } else if (nj <= 32) {
    scatter_class_regs<32>(i, X, ldx, c0, nj, HW, ldw, s);
  } else {
    for (int64_t c = c0; c < c1; ++c) s += X[i + c * ldx];
    const double mj = s / (double)nj;
    for (int64_t c = c0; c < c1; ++c) HW[i + c * ldw] = X[i + c * ldx] - mj;
  }
  HB[i + j * ldb] = s;
}

__global__ __launch_bounds__(256) void scatter_between_kernel(int64_t d, int64_t n, int64_t k,
                                                              const int64_t* __restrict__ offs,
                                                              double* __restrict__ HB,
                                                              int64_t ldb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= d) return;
  double total = 0.0;
  for (int64_t j = 0; j < k; ++j) total += HB[i + j * ldb];
  const double mu = total / (double)n;  // sample-weighted global centroid
  for (int64_t j = 0; j < k; ++j) {
    const double nj = (double)(offs[j + 1] - offs[j]);
    HB[i + j * ldb] = sqrt(nj) * (HB[i + j * ldb] / nj - mu);
  }
}

// With a flag, flag[0] |= 1 when an entry read is NaN or Inf (the pass that
// copies the factor also checks it).
template <typename TP>
__global__ __launch_bounds__(256) void pack_kernel(int64_t d, int64_t ldp, const double* __restrict__ H,
                                                   int64_t ldh, TP* __restrict__ P, int64_t col0,
                                                   int* flag) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  const double v = (r < d) ? H[r + c * ldh] : 0.0;
  if (flag != nullptr && __any(!isfinite(v)) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
  if (r >= ldp) return;
  P[r + (col0 + c) * ldp] = from_f64<TP>(v);
}

// FP8 storage: per-column scale max_r |P[r, j]| / 448 (1 for a zero
// column), so that the largest entry of every column maps to the largest
// finite E4M3 value.  One workgroup per column.
__global__ __launch_bounds__(256) void fp8_scale_kernel(int64_t d, const double* __restrict__ P,
                                                        int64_t ldp, double* __restrict__ scale) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  double mx = 0.0;
  for (int64_t r = threadIdx.x; r < d; r += 256) mx = fmax(mx, fabs(P[r + c * ldp]));
  for (int m = 32; m >= 1; m >>= 1) mx = fmax(mx, __shfl_xor(mx, m));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double t = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
    scale[c] = (t > 0.0) ? t / 448.0 : 1.0;
  }
}

__global__ __launch_bounds__(256) void pack_fp8_kernel(int64_t d, int64_t ldp,
                                                       const double* __restrict__ P,
                                                       const double* __restrict__ scale,
                                                       uint8_t* __restrict__ P8) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= ldp) return;
  P8[r + c * ldp] = (r < d) ? fp8e4m3_encode(P[r + c * ldp] / scale[c]) : (uint8_t)0;
}

__global__ __launch_bounds__(256) void nonfinite_kernel(int64_t d, int64_t cols, const double* __restrict__ H,
                                                        int64_t ldh, int* flag) {
  const int64_t total = d * cols;
  int bad = 0;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t c = e / d, r = e - c * d;
    const double v = H[r + c * ldh];
    bad |= !isfinite(v);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// SplitMix64 finaliser (Steele, Lea, Flood, OOPSLA 2014) used as a counter hash.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9e3779b97f4a7c15ull;
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  return z ^ (z >> 31);
}

__global__ __launch_bounds__(256) void randn_kernel(const RandnArgs* __restrict__ arr, RandnArgs one) {
  const RandnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t d = a.d, b = a.b, ldv = a.ldv;
  const uint64_t seed = a.seed;
  double* __restrict__ V = a.V;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= d * b) return;
  const int64_t c = e / d, r = e - c * d;
  const uint64_t base = seed * 0xd1342543de82ef95ull;
  const uint64_t z1 = splitmix64(base + 2ull * (uint64_t)e);
  const uint64_t z2 = splitmix64(base + 2ull * (uint64_t)e + 1ull);
  const double u1 = ((double)(z1 >> 11) + 1.0) * 0x1.0p-53;  // (0, 1]
  const double u2 = (double)(z2 >> 11) * 0x1.0p-53;          // [0, 1)
  V[r + c * ldv] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);  // Box-Muller
}

template <typename TS, typename TD>
__global__ __launch_bounds__(256) void copy2d_kernel(const Copy2dArgs* __restrict__ arr, Copy2dArgs one) {
  const Copy2dArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= a.rows || c >= a.cols) return;
  ((TD*)a.dst)[r + c * a.ldd] = from_f64<TD>(to_f64<TS>(((const TS*)a.src)[r + c * a.lds]));
}

// Weights of a core G = V diag(f) V^T of the exponential exp(c H H^T)
// scaled by e^{-shift}:  f(l) = e^{-shift} (e^{c l} - 1) / l,  f(0) = c e^{-shift}.
__global__ __launch_bounds__(256) void core_weights_kernel(int64_t n, const double* __restrict__ lam,
                                                           double c, double shift,
                                                           double* __restrict__ f) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double l = lam[i];
  const double cl = c * l;
  double v;
  if (fabs(l) < 1e-300) {
    v = c * exp(-shift);
  } else if (cl <= 1.0) {
    v = exp(-shift) * expm1(cl) / l;
  } else {
    v = (exp(cl - shift) - exp(-shift)) / l;
  }
  f[i] = v;
}

// One workgroup per column: make the largest-magnitude entry positive
// (ties: the smallest row index).
__global__ __launch_bounds__(1024) void sign_fix_kernel(const SignArgs* __restrict__ arr, SignArgs one) {
  const SignArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if ((int64_t)blockIdx.x >= a.t) return;
  const int64_t d = a.d;
  __shared__ double sv[1024];
  __shared__ int64_t si[1024];
  double* x = a.X + blockIdx.x * a.ldx;
  double best = -1.0;
  int64_t bi = 0;
  const int64_t nt = blockDim.x;
  // eight loads in flight per thread; each thread visits its rows in
  // increasing order, so ties keep the smallest index
  for (int64_t r0 = threadIdx.x; r0 < d; r0 += 8 * nt) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (r0 + u * nt < d) ? fabs(x[r0 + u * nt]) : -1.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (v[u] > best) { best = v[u]; bi = r0 + u * nt; }
  }
  sv[threadIdx.x] = best;
  si[threadIdx.x] = bi;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      const double a = sv[threadIdx.x + s];
      const int64_t ai = si[threadIdx.x + s];
      if (a > sv[threadIdx.x] || (a == sv[threadIdx.x] && ai < si[threadIdx.x])) {
        sv[threadIdx.x] = a;
        si[threadIdx.x] = ai;
      }
    }
    __syncthreads();
  }
  const bool flip = x[si[0]] < 0.0;  // uniform across the workgroup
  __syncthreads();  // every thread has read the pivot before any entry changes
  if (!flip) return;
  for (int64_t r0 = threadIdx.x; r0 < d; r0 += 8 * nt) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = (r0 + u * nt < d) ? x[r0 + u * nt] : 0.0;
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (r0 + u * nt < d) x[r0 + u * nt] = -v[u];
  }
}

__global__ __launch_bounds__(256) void fill_kernel(const FillArgs* __restrict__ arr, FillArgs one) {
  const FillArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < a.count) a.dst[e] = a.v;
}

__global__ __launch_bounds__(256) void fill_i32_kernel(const FillI32Args* __restrict__ arr, FillI32Args one) {
  const FillI32Args a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e < a.count) a.dst[e] = a.v;
}

__global__ __launch_bounds__(256) void symmetrize_kernel(const SymArgs* __restrict__ arr, SymArgs one) {
  const SymArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= a.m || c >= a.m) return;
  a.T[r + c * a.ldt] = 0.5 * (a.H[r + c * a.ldh] + a.H[c + r * a.ldh]);
}

__global__ __launch_bounds__(64) void ritz_estimates_kernel(const RitzEstArgs* __restrict__ arr,
                                                            RitzEstArgs one) {
  const RitzEstArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t m = a.m, b = a.b, lds = a.lds, ldbm = a.ldbm;
  const double* __restrict__ w = a.w;
  const double* __restrict__ S = a.S;
  const double* __restrict__ Bm = a.Bm;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.cnt) return;
  double* __restrict__ th = a.th;
  double* __restrict__ res = a.res;
  const int64_t col = m - 1 - i;
  double acc = 0.0;
  for (int64_t r = 0; r < b; ++r) {
    double s = 0.0;
    for (int64_t q = 0; q < b; ++q) s += Bm[r + q * ldbm] * S[(m - b + q) + col * lds];
    acc += s * s;
  }
  th[i] = w[col];
  res[i] = sqrt(acc);
}

__global__ __launch_bounds__(256) void gather_desc_kernel(const GatherArgs* __restrict__ arr, GatherArgs one) {
  const GatherArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t i = blockIdx.y;
  if (r >= a.m || i >= a.cnt) return;
  a.Sd[r * a.ldsd + i] = a.S[r + (a.m - 1 - i) * a.lds];
}

__global__ void flag_fold_kernel(const FlagArgs* __restrict__ arr, FlagArgs one) {
  int* flags = (arr != nullptr ? arr[blockIdx.z] : one).flags;
  if (threadIdx.x == 0) {
    flags[1] |= flags[0];
    flags[0] = 0;
  }
}

// R[:, c] = MY[:, c] - theta_c Y[:, c] (stored when R is not null) and
// res[c] = ||R[:, c]||_2, one workgroup of 1024 threads per column.  With
// 16-byte aligned columns each thread takes four row pairs a round, all
// loads issued before the arithmetic, so that a compute unit keeps enough
// loads in flight; fixed-order block sum.
__global__ __launch_bounds__(1024) void ritz_residual_kernel(const ResidArgs* __restrict__ arr,
                                                             ResidArgs one) {
  typedef double d2 __attribute__((ext_vector_type(2)));
  const ResidArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t c = blockIdx.x;
  if (c >= a.t) return;
  const int64_t d = a.d;
  const double* __restrict__ my = a.MY + c * a.ldmy;
  const double* __restrict__ y = a.Y + c * a.ldy;
  double* __restrict__ rr = (a.R != nullptr) ? a.R + c * a.ldr : nullptr;
  __shared__ double red[16];
  const double th = a.theta[c];
  const bool vec = ((uintptr_t)my % 16 == 0) && ((uintptr_t)y % 16 == 0) &&
                   (rr == nullptr || (uintptr_t)rr % 16 == 0);
  double acc = 0.0;
  int64_t r0 = 0;
  if (vec) {
    const int64_t np = d / 2;
    for (int64_t p0 = 0; p0 < np; p0 += 4 * 1024) {
      d2 xm[4], xy[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t p = p0 + threadIdx.x + 1024 * u;
        const int64_t pc = (p < np) ? p : 0;
        xm[u] = *(const d2*)(my + 2 * pc);
        xy[u] = *(const d2*)(y + 2 * pc);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t p = p0 + threadIdx.x + 1024 * u;
        if (p < np) {
          d2 v;
          v.x = xm[u].x - th * xy[u].x;
          v.y = xm[u].y - th * xy[u].y;
          if (rr != nullptr) *(d2*)(rr + 2 * p) = v;
          acc += v.x * v.x + v.y * v.y;
        }
      }
    }
    r0 = 2 * np;
  }
  for (int64_t r = r0 + threadIdx.x; r < d; r += blockDim.x) {
    const double v = my[r] - th * y[r];
    if (rr != nullptr) rr[r] = v;
    acc += v * v;
  }
  acc = block_sum(acc, red);
  if (threadIdx.x == 0) a.res[c] = sqrt(acc);
}

// out[i] = w[n - 1 - i] for i < cnt (ascending eigenvalues to descending).
__global__ __launch_bounds__(256) void desc_values_kernel(const DescArgs* __restrict__ arr, DescArgs one) {
  const DescArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < a.cnt) a.out[i] = a.w[a.n - 1 - i];
}

__global__ __launch_bounds__(256) void restart_coupling_kernel(const CouplingArgs* __restrict__ arr,
                                                               CouplingArgs one) {
  const CouplingArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t m = a.m, b = a.b, kk = a.kk, ldbm = a.ldbm, ldsd = a.ldsd, ldh = a.ldh;
  const double* __restrict__ Bm = a.Bm;
  const double* __restrict__ Sd = a.Sd;
  double* __restrict__ Hn = a.Hn;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= b * kk) return;
  const int64_t c = e / b, r = e - c * b;
  double s = 0.0;
  for (int64_t q = 0; q < b; ++q) s += Bm[r + q * ldbm] * Sd[(m - b + q) * ldsd + c];
  Hn[(kk + r) + c * ldh] = s;
}

__global__ __launch_bounds__(256) void copy_block_kernel(int64_t rows, int64_t cols, double alpha,
                                                         const double* __restrict__ S, int64_t lds,
                                                         bool trans, double* __restrict__ D,
                                                         int64_t ldd) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int64_t c = e / rows, r = e - c * rows;
  D[r + c * ldd] = alpha * (trans ? S[c + r * lds] : S[r + c * lds]);
}

__global__ __launch_bounds__(256) void set_diag_kernel(const SetDiagArgs* __restrict__ arr, SetDiagArgs one) {
  const SetDiagArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < a.cnt) a.D[i + i * a.ldd] = a.v[i];
}

// One wave per column (lanes over rows, coalesced), loads batched by eight;
// the column sums meet in *out through an atomic maximum on their bit
// patterns (non-negative doubles order like their unsigned 64-bit patterns).
// *out must hold +0.0 before the launch.
__global__ __launch_bounds__(256) void norm1_kernel(int64_t n, const double* __restrict__ A,
                                                    int64_t lda, double* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int64_t j = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= n) return;
  const double* col = A + j * lda;
  double s = 0.0;
  for (int64_t i0 = lane; i0 < n; i0 += 64 * 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t i = i0 + 64 * u;
      v[u] = (i < n) ? fabs(col[i]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  s = wave_sum(s);
  if (lane == 0)
    atomicMax((unsigned long long*)out, (unsigned long long)__double_as_longlong(s));
}

__global__ __launch_bounds__(256) void lincomb_kernel(int64_t n, double a0, double a1,
                                                      const double* __restrict__ X1, double a2,
                                                      const double* __restrict__ X2, double a3,
                                                      const double* __restrict__ X3, int64_t ldx,
                                                      double* __restrict__ C, int64_t ldc) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= n * n) return;
  const int64_t c = e / n, r = e - c * n;
  double v = (r == c) ? a0 : 0.0;
  v += a1 * X1[r + c * ldx];
  if (a2 != 0.0) v += a2 * X2[r + c * ldx];
  if (a3 != 0.0) v += a3 * X3[r + c * ldx];
  C[r + c * ldc] = v;
}

inline unsigned nblk(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

hipError_t launch_norm1(int64_t n, const double* A, int64_t lda, double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const hipError_t e = launch_fill(1, 0.0, out, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(norm1_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, A, lda, out);
  return hipGetLastError();
}

hipError_t launch_lincomb(int64_t n, double a0, double a1, const double* X1, double a2,
                          const double* X2, double a3, const double* X3, int64_t ldx,
                          double* C, int64_t ldc, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(lincomb_kernel, dim3(nblk(n * n)), dim3(256), 0, s, n, a0, a1, X1, a2, X2,
                     a3, X3, ldx, C, ldc);
  return hipGetLastError();
}

hipError_t launch_copy_block(int64_t rows, int64_t cols, double alpha, const double* src,
                             int64_t lds, bool trans, double* dst, int64_t ldd, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(copy_block_kernel, dim3(nblk(rows * cols)), dim3(256), 0, s, rows, cols,
                     alpha, src, lds, trans, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_scatter(int64_t d, int64_t n, int64_t k, const double* X, int64_t ldx,
                          const int64_t* offsets, double* H_W, int64_t ldw, double* H_B,
                          int64_t ldb, hipStream_t s) {
  hipLaunchKernelGGL(scatter_class_kernel, dim3(nblk(d), (unsigned)k), dim3(256), 0, s, d, X, ldx,
                     offsets, H_W, ldw, H_B, ldb);
  hipLaunchKernelGGL(scatter_between_kernel, dim3(nblk(d)), dim3(256), 0, s, d, n, k, offsets, H_B,
                     ldb);
  return hipGetLastError();
}

hipError_t launch_pack(int64_t d, int64_t ldp, int64_t cols, const double* H, int64_t ldh,
                       void* P, DT pdt, int64_t col0, hipStream_t s, int* flag) {
  if (cols <= 0) return hipSuccess;
  dim3 g(nblk(ldp), (unsigned)cols);
  if (pdt == DT::F64)
    hipLaunchKernelGGL(pack_kernel<double>, g, dim3(256), 0, s, d, ldp, H, ldh, (double*)P, col0,
                       flag);
  else if (pdt == DT::F32)
    hipLaunchKernelGGL(pack_kernel<float>, g, dim3(256), 0, s, d, ldp, H, ldh, (float*)P, col0,
                       flag);
  else
    hipLaunchKernelGGL(pack_kernel<bf16_t>, g, dim3(256), 0, s, d, ldp, H, ldh, (bf16_t*)P, col0,
                       flag);
  return hipGetLastError();
}

hipError_t launch_pack_fp8(int64_t d, int64_t ldp, int64_t cols, const double* P64,
                           double* scale, void* P8, hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(fp8_scale_kernel, dim3((unsigned)cols), dim3(256), 0, s, d, P64, ldp, scale);
  hipLaunchKernelGGL(pack_fp8_kernel, dim3(nblk(ldp), (unsigned)cols), dim3(256), 0, s, d, ldp,
                     P64, (const double*)scale, (uint8_t*)P8);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void scale_cols_kernel(int64_t rows, const double* __restrict__ src,
                                                         int64_t lds, const double* __restrict__ w,
                                                         int p, double* __restrict__ dst,
                                                         int64_t ldd) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t c = blockIdx.y;
  if (r >= rows) return;
  const double f = sqrt(w[c]);
  dst[r + c * ldd] = (p > 0) ? src[r + c * lds] * f : src[r + c * lds] / f;
}

hipError_t launch_scale_cols(int64_t rows, int64_t cols, const double* src, int64_t lds,
                             const double* w, int p, double* dst, int64_t ldd, hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_cols_kernel, dim3(nblk(rows), (unsigned)cols), dim3(256), 0, s, rows,
                     src, lds, w, p, dst, ldd);
  return hipGetLastError();
}

hipError_t launch_nonfinite(int64_t d, int64_t cols, const double* H, int64_t ldh, int* flag,
                            hipStream_t s) {
  int64_t total = d * cols;
  unsigned g = (unsigned)std::min<int64_t>(2048, (total + 255) / 256);
  if (g == 0) return hipSuccess;
  hipLaunchKernelGGL(nonfinite_kernel, dim3(g), dim3(256), 0, s, d, cols, H, ldh, flag);
  return hipGetLastError();
}

hipError_t launch_core_weights(int64_t n, const double* lam, double c, double shift, double* f,
                               hipStream_t s) {
  hipLaunchKernelGGL(core_weights_kernel, dim3(nblk(n)), dim3(256), 0, s, n, lam, c, shift, f);
  return hipGetLastError();
}

// ---- multi-problem launchers (count == 1: arguments by value) -------------

hipError_t launch_randn_multi(int count, const RandnArgs* host, const RandnArgs* dev,
                              hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, nblk(host[p].d * host[p].b));
  if (x == 0) return hipSuccess;
  const RandnArgs* arr;
  RandnArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(randn_kernel, dim3((unsigned)x, 1, (unsigned)count), dim3(256), 0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_copy2d_multi(int count, const Copy2dArgs* host, const Copy2dArgs* dev, DT sdt,
                               DT ddt, hipStream_t s) {
  int64_t x = 0, y = 0;
  for (int p = 0; p < count; ++p) {
    if (host[p].rows <= 0 || host[p].cols <= 0) continue;
    x = std::max<int64_t>(x, nblk(host[p].rows));
    y = std::max<int64_t>(y, host[p].cols);
  }
  if (x == 0) return hipSuccess;
  const Copy2dArgs* arr;
  Copy2dArgs one;
  pick(count, host, dev, &arr, &one);
  dim3 g((unsigned)x, (unsigned)y, (unsigned)count);
  if (sdt == DT::F64 && ddt == DT::F64)
    hipLaunchKernelGGL((copy2d_kernel<double, double>), g, dim3(256), 0, s, arr, one);
  else if (sdt == DT::F64 && ddt == DT::F32)
    hipLaunchKernelGGL((copy2d_kernel<double, float>), g, dim3(256), 0, s, arr, one);
  else if (sdt == DT::F32 && ddt == DT::F64)
    hipLaunchKernelGGL((copy2d_kernel<float, double>), g, dim3(256), 0, s, arr, one);
  else if (sdt == DT::F32 && ddt == DT::F32)
    hipLaunchKernelGGL((copy2d_kernel<float, float>), g, dim3(256), 0, s, arr, one);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_sign_fix_multi(int count, const SignArgs* host, const SignArgs* dev,
                                 hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, host[p].t);
  if (x == 0) return hipSuccess;
  const SignArgs* arr;
  SignArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(sign_fix_kernel, dim3((unsigned)x, 1, (unsigned)count), dim3(1024), 0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_fill_multi(int count, const FillArgs* host, const FillArgs* dev, hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, nblk(host[p].count));
  if (x == 0) return hipSuccess;
  const FillArgs* arr;
  FillArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(fill_kernel, dim3((unsigned)x, 1, (unsigned)count), dim3(256), 0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_fill_i32_multi(int count, const FillI32Args* host, const FillI32Args* dev,
                                 hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, nblk(host[p].count));
  if (x == 0) return hipSuccess;
  const FillI32Args* arr;
  FillI32Args one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(fill_i32_kernel, dim3((unsigned)x, 1, (unsigned)count), dim3(256), 0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_symmetrize_multi(int count, const SymArgs* host, const SymArgs* dev,
                                   hipStream_t s) {
  int64_t x = 0, y = 0;
  for (int p = 0; p < count; ++p) {
    x = std::max<int64_t>(x, nblk(host[p].m));
    y = std::max<int64_t>(y, host[p].m);
  }
  if (x == 0) return hipSuccess;
  const SymArgs* arr;
  SymArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(symmetrize_kernel, dim3((unsigned)x, (unsigned)y, (unsigned)count), dim3(256),
                     0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_ritz_estimates_multi(int count, const RitzEstArgs* host, const RitzEstArgs* dev,
                                       hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, nblk(host[p].cnt, 64));
  if (x == 0) return hipSuccess;
  const RitzEstArgs* arr;
  RitzEstArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(ritz_estimates_kernel, dim3((unsigned)x, 1, (unsigned)count), dim3(64), 0, s,
                     arr, one);
  return hipGetLastError();
}

hipError_t launch_gather_desc_multi(int count, const GatherArgs* host, const GatherArgs* dev,
                                    hipStream_t s) {
  int64_t x = 0, y = 0;
  for (int p = 0; p < count; ++p) {
    x = std::max<int64_t>(x, nblk(host[p].m));
    y = std::max<int64_t>(y, host[p].cnt);
  }
  if (x == 0 || y == 0) return hipSuccess;
  const GatherArgs* arr;
  GatherArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(gather_desc_kernel, dim3((unsigned)x, (unsigned)y, (unsigned)count), dim3(256),
                     0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_flag_fold_multi(int count, const FlagArgs* host, const FlagArgs* dev,
                                  hipStream_t s) {
  if (count < 1) return hipSuccess;
  const FlagArgs* arr;
  FlagArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(flag_fold_kernel, dim3(1, 1, (unsigned)count), dim3(64), 0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_ritz_residual_multi(int count, const ResidArgs* host, const ResidArgs* dev,
                                      hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, host[p].t);
  if (x == 0) return hipSuccess;
  const ResidArgs* arr;
  ResidArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(ritz_residual_kernel, dim3((unsigned)x, 1, (unsigned)count), dim3(1024), 0, s,
                     arr, one);
  return hipGetLastError();
}

hipError_t launch_desc_values_multi(int count, const DescArgs* host, const DescArgs* dev,
                                    hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, nblk(host[p].cnt));
  if (x == 0) return hipSuccess;
  const DescArgs* arr;
  DescArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(desc_values_kernel, dim3((unsigned)x, 1, (unsigned)count), dim3(256), 0, s,
                     arr, one);
  return hipGetLastError();
}

hipError_t launch_restart_coupling_multi(int count, const CouplingArgs* host,
                                         const CouplingArgs* dev, hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, nblk(host[p].b * host[p].kk));
  if (x == 0) return hipSuccess;
  const CouplingArgs* arr;
  CouplingArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(restart_coupling_kernel, dim3((unsigned)x, 1, (unsigned)count), dim3(256), 0,
                     s, arr, one);
  return hipGetLastError();
}

hipError_t launch_set_diag_multi(int count, const SetDiagArgs* host, const SetDiagArgs* dev,
                                 hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, nblk(host[p].cnt));
  if (x == 0) return hipSuccess;
  const SetDiagArgs* arr;
  SetDiagArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(set_diag_kernel, dim3((unsigned)x, 1, (unsigned)count), dim3(256), 0, s, arr,
                     one);
  return hipGetLastError();
}

// ---- single-problem wrappers ------------------------------------------------
hipError_t launch_randn(int64_t d, int64_t b, uint64_t seed, double* V, int64_t ldv,
                        hipStream_t s) {
  RandnArgs a{d, b, ldv, seed, V};
  return launch_randn_multi(1, &a, nullptr, s);
}
hipError_t launch_copy2d(int64_t rows, int64_t cols, const void* src, DT sdt, int64_t lds,
                         void* dst, DT ddt, int64_t ldd, hipStream_t s) {
  Copy2dArgs a{rows, cols, lds, ldd, src, dst};
  return launch_copy2d_multi(1, &a, nullptr, sdt, ddt, s);
}
namespace {

// One workgroup per testing sample: its projection in LDS, the training
// projections split over the threads (each keeps its first minimum, rows in
// increasing order), then a fixed-order reduction that keeps the smaller
// index on equal distances.
constexpr int NNC_TMAX = 1024;
__global__ __launch_bounds__(256) void nn_classify_kernel(int64_t n_train, int64_t t,
                                                          const double* __restrict__ Ptr,
                                                          const double* __restrict__ Pte,
                                                          const int32_t* __restrict__ labels,
                                                          int32_t* __restrict__ pred,
                                                          int64_t* __restrict__ idx,
                                                          double* __restrict__ dist) {
  __shared__ double q[NNC_TMAX];
  __shared__ double bd[256];
  __shared__ int64_t bi[256];
  const int64_t j = blockIdx.x;
  const int tid = threadIdx.x;
  for (int64_t k = tid; k < t; k += 256) q[k] = Pte[j * t + k];
  __syncthreads();
  double best = INFINITY;
  int64_t besti = -1;
  for (int64_t i = tid; i < n_train; i += 256) {
    const double* p = Ptr + i * t;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t k = 0;
    for (; k + 4 <= t; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const double df = p[k + u] - q[k + u];
        acc[u] = fma(df, df, acc[u]);
      }
    }
    for (; k < t; ++k) {
      const double df = p[k] - q[k];
      acc[0] = fma(df, df, acc[0]);
    }
    const double d2 = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    if (d2 < best) {
      best = d2;
      besti = i;
    }
  }
  bd[tid] = best;
  bi[tid] = besti;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
      const double o = bd[tid + h];
      const int64_t oi = bi[tid + h];
      if (oi >= 0 && (bi[tid] < 0 || o < bd[tid] || (o == bd[tid] && oi < bi[tid]))) {
        bd[tid] = o;
        bi[tid] = oi;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {  // (no index: every distance was NaN)
    const int64_t b = bi[0];
    idx[j] = b;
    pred[j] = (b >= 0) ? labels[b] : -1;
    dist[j] = (b >= 0) ? sqrt(bd[0]) : NAN;
  }
}

}  // namespace

hipError_t launch_nn_classify(int64_t n_train, int64_t n_test, int64_t t, const double* Ptr,
                              const double* Pte, const int32_t* labels, int32_t* pred,
                              int64_t* idx, double* dist, hipStream_t s) {
  if (n_train < 1 || n_test < 1 || t < 1 || t > NNC_TMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(nn_classify_kernel, dim3((unsigned)n_test), dim3(256), 0, s, n_train, t,
                     Ptr, Pte, labels, pred, idx, dist);
  return hipGetLastError();
}

hipError_t launch_sign_fix(int64_t d, int64_t t, double* X, int64_t ldx, hipStream_t s) {
  SignArgs a{d, t, ldx, X};
  return launch_sign_fix_multi(1, &a, nullptr, s);
}
hipError_t launch_fill(int64_t count, double value, double* dst, hipStream_t s) {
  FillArgs a{count, value, dst};
  return launch_fill_multi(1, &a, nullptr, s);
}
hipError_t launch_fill_i32(int64_t count, int value, int* dst, hipStream_t s) {
  FillI32Args a{count, value, dst};
  return launch_fill_i32_multi(1, &a, nullptr, s);
}
hipError_t launch_symmetrize(int64_t m, const double* H, int64_t ldh, double* T, int64_t ldt,
                             hipStream_t s) {
  SymArgs a{m, ldh, ldt, H, T};
  return launch_symmetrize_multi(1, &a, nullptr, s);
}
hipError_t launch_ritz_estimates(int64_t m, int64_t b, int64_t cnt, const double* w,
                                 const double* S, int64_t lds, const double* Bm, int64_t ldbm,
                                 double* out_theta, double* out_res, hipStream_t s) {
  RitzEstArgs a{m, b, cnt, lds, ldbm, w, S, Bm, out_theta, out_res};
  return launch_ritz_estimates_multi(1, &a, nullptr, s);
}
hipError_t launch_gather_desc(int64_t m, int64_t cnt, const double* S, int64_t lds, double* Sd,
                              int64_t ldsd, hipStream_t s) {
  GatherArgs a{m, cnt, lds, ldsd, S, Sd};
  return launch_gather_desc_multi(1, &a, nullptr, s);
}
hipError_t launch_flag_fold(int* flags, hipStream_t s) {
  FlagArgs a{flags};
  return launch_flag_fold_multi(1, &a, nullptr, s);
}
hipError_t launch_ritz_residual(int64_t d, int64_t t, const double* MY, int64_t ldmy,
                                const double* Y, int64_t ldy, const double* theta, double* R,
                                int64_t ldr, double* res, hipStream_t s) {
  ResidArgs a{d, t, ldmy, ldy, ldr, MY, Y, theta, R, res};
  return launch_ritz_residual_multi(1, &a, nullptr, s);
}
hipError_t launch_desc_values(int64_t cnt, const double* w, int64_t n, double* out,
                              hipStream_t s) {
  DescArgs a{cnt, n, w, out};
  return launch_desc_values_multi(1, &a, nullptr, s);
}
hipError_t launch_restart_coupling(int64_t m, int64_t b, int64_t kk, const double* Bm,
                                   int64_t ldbm, const double* Sd, int64_t ldsd, double* Hn,
                                   int64_t ldh, hipStream_t s) {
  CouplingArgs a{m, b, kk, ldbm, ldsd, ldh, Bm, Sd, Hn};
  return launch_restart_coupling_multi(1, &a, nullptr, s);
}
hipError_t launch_set_diag(int64_t cnt, const double* v, double* dst, int64_t ldd, hipStream_t s) {
  SetDiagArgs a{cnt, ldd, v, dst};
  return launch_set_diag_multi(1, &a, nullptr, s);
}

}  // namespace eda
