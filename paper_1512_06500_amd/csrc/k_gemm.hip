// Small dense FP64 products: general GEMM for the cores (n x n and n x k
// factors of the exponentials) on the matrix cores, and the Gram matrix
// P^T P of the scatter factors (register-tiled FMA kernel: 64 x 64 output
// tiles, 256 threads, 4 x 4 outputs per thread, K staged through LDS in
// slices of 16).
#include "common.h"

namespace eda {

namespace {

constexpr int GT = 64;   // tile edge
constexpr int GK = 16;   // K slice

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int MT = 32;  // output tile edge of the matrix-core GEMM
constexpr int MK = 64;  // K slice

// C = alpha op(A) diag(dk) op(B) + beta C on the matrix cores: a 256-thread
// workgroup owns a 32 x 32 tile of C, each wave one 16 x 16 block of it,
// accumulated by v_mfma_f64_16x16x4f64 over K slices of 64 staged in LDS.
// The next slice is loaded into registers while the current one is
// multiplied, so a slice costs one memory round trip at most (the products
// of the cores have K = n or k, a few slices).  Operand lane layout:
// A(i, k) at lane i + 16 k, B(k, j) at lane j + 16 k; accumulator element v
// of lane l is C(4 v + l / 16, l % 16).
__global__ __launch_bounds__(256) void gemm_kernel(bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                                                   double alpha, const double* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ dk,
                                                   const double* __restrict__ B, int64_t ldb,
                                                   double beta, double* __restrict__ C,
                                                   int64_t ldc) {
  __shared__ double As[MT][MK + 1];  // op(A)(i, k)
  __shared__ double Bs[MK][MT + 1];  // op(B)(k, j)
  constexpr int NL = MT * MK / 256;  // elements of each tile per thread
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int64_t i0 = blockIdx.x * (int64_t)MT, j0 = blockIdx.y * (int64_t)MT;
  const int bi = (wid >> 1) * 16, bj = (wid & 1) * 16;
  // element q of this thread: (ii, kk) of op(A) and (kb, jj) of op(B), with
  // consecutive threads on consecutive addresses
  auto a_pos = [&](int q, int& ii, int& kk) {
    const int e = tid + q * 256;
    if (!ta) { ii = e & (MT - 1); kk = e / MT; } else { kk = e & (MK - 1); ii = e / MK; }
  };
  auto b_pos = [&](int q, int& kb, int& jj) {
    const int e = tid + q * 256;
    if (!tb) { kb = e & (MK - 1); jj = e / MK; } else { jj = e & (MT - 1); kb = e / MT; }
  };
  double ra[NL], rb[NL];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      int ii, kk, kb, jj;
      a_pos(q, ii, kk);
      b_pos(q, kb, jj);
      const int64_t gi = i0 + ii, gk = k0 + kk, gj = j0 + jj, gk2 = k0 + kb;
      double v = 0.0, w = 0.0;
      if (gi < m && gk < k) {
        v = ta ? A[gk + gi * lda] : A[gi + gk * lda];
        if (dk != nullptr) v *= dk[gk];
      }
      if (gj < n && gk2 < k) w = tb ? B[gj + gk2 * ldb] : B[gk2 + gj * ldb];
      ra[q] = v;
      rb[q] = w;
    }
  };
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  if (k > 0) load(0);
  for (int64_t k0 = 0; k0 < k; k0 += MK) {
    __syncthreads();  // the previous slice has been read
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      int ii, kk, kb, jj;
      a_pos(q, ii, kk);
      b_pos(q, kb, jj);
      As[ii][kk] = ra[q];
      Bs[kb][jj] = rb[q];
    }
    __syncthreads();
    if (k0 + MK < k) load(k0 + MK);  // in flight during the products below
    const int kl = (k - k0 < MK) ? (int)(k - k0) : MK;
#pragma unroll
    for (int ks = 0; ks < MK; ks += 4) {
      if (ks >= kl) break;  // uniform
      const double a = As[bi + (lane & 15)][ks + (lane >> 4)];
      const double b = Bs[ks + (lane >> 4)][bj + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
  const int64_t gj = j0 + bj + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t gi = i0 + bi + 4 * v + (lane >> 4);
    if (gi >= m || gj >= n) continue;
    double* cp = C + gi + gj * ldc;
    *cp = (beta == 0.0 ? 0.0 : beta * *cp) + alpha * acc[v];
  }
}

// Gram partials over one row chunk for one lower-triangle tile (ti >= tj).
template <typename TP>
__global__ __launch_bounds__(256) void gram_partial_kernel(int64_t d, int64_t N,
                                                           const TP* __restrict__ P, int64_t ldp,
                                                           double* __restrict__ part,
                                                           int64_t rows_per_chunk) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  // blockIdx.x enumerates lower-triangle tiles, blockIdx.y row chunks
  int64_t t = blockIdx.x, ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int64_t tj = t - ti * (ti + 1) / 2;
  const int64_t i0 = ti * GT, j0 = tj * GT;
  const int64_t c = blockIdx.y;
  const int64_t r0 = c * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk < d) ? r0 + rows_per_chunk : d;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

  for (int64_t k0 = r0; k0 < r1; k0 += GK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      const int kk = e & 15, ii = e >> 4;
      const int64_t gk = k0 + kk;
      const int64_t gi = i0 + ii, gj = j0 + ii;
      As[kk][ii] = (gi < N && gk < r1) ? to_f64<TP>(P[gk + gi * ldp]) : 0.0;
      Bs[kk][ii] = (gj < N && gk < r1) ? to_f64<TP>(P[gk + gj * ldp]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = As[kk][tx + 16 * q];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = Bs[kk][ty + 16 * q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
    __syncthreads();
  }
  double* pc = part + c * N * N;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int64_t gi = i0 + tx + 16 * p;
    if (gi >= N) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t gj = j0 + ty + 16 * q;
      if (gj >= N) continue;
      pc[gi + gj * N] = acc[p][q];
    }
  }
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(int64_t N, int64_t chunks,
                                                          const double* __restrict__ part,
                                                          double* __restrict__ G, int64_t ldg) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= N * N) return;
  const int64_t j = e / N, i = e - j * N;
  // read from the lower-triangle tile that holds (i, j) or its mirror
  const bool lower = (i / GT) >= (j / GT);
  const int64_t src = lower ? (i + j * N) : (j + i * N);
  double s = 0.0;
  for (int64_t c = 0; c < chunks; ++c) s += part[c * N * N + src];
  G[i + j * ldg] = s;
}

void gram_geometry(int64_t d, int64_t N, int64_t* chunks, int64_t* rows) {
  const int64_t T = (N + GT - 1) / GT;
  const int64_t tiles = T * (T + 1) / 2;
  int64_t c = (1024 + tiles - 1) / tiles;
  const int64_t cmax = std::max<int64_t>(1, (d + 255) / 256);
  c = std::max<int64_t>(1, std::min(c, cmax));
  int64_t rp = (d + c - 1) / c;
  rp = ((rp + GK - 1) / GK) * GK;
  *rows = rp;
  *chunks = (d + rp - 1) / rp;
}

}  // namespace

hipError_t launch_gemm(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double alpha,
                       const double* A, int64_t lda, const double* dk, const double* B,
                       int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  dim3 g((unsigned)((m + MT - 1) / MT), (unsigned)((n + MT - 1) / MT));
  hipLaunchKernelGGL(gemm_kernel, g, dim3(256), 0, s, ta, tb, m, n, k, alpha, A, lda, dk, B, ldb,
                     beta, C, ldc);
  return hipGetLastError();
}

int64_t gram_chunks(int64_t d, int64_t N) {
  int64_t c, r;
  gram_geometry(d, N, &c, &r);
  return c;
}

hipError_t launch_gram_partial(int64_t d, int64_t N, const void* P, DT pdt, int64_t ldp,
                               double* part, int64_t chunks, hipStream_t s) {
  int64_t c, rows;
  gram_geometry(d, N, &c, &rows);
  if (c != chunks) return hipErrorInvalidValue;
  const int64_t T = (N + GT - 1) / GT;
  dim3 g((unsigned)(T * (T + 1) / 2), (unsigned)chunks);
  if (pdt == DT::F64)
    hipLaunchKernelGGL(gram_partial_kernel<double>, g, dim3(256), 0, s, d, N, (const double*)P,
                       ldp, part, rows);
  else
    hipLaunchKernelGGL(gram_partial_kernel<float>, g, dim3(256), 0, s, d, N, (const float*)P, ldp,
                       part, rows);
  return hipGetLastError();
}

hipError_t launch_gram_reduce(int64_t N, int64_t chunks, const double* part, double* G,
                              int64_t ldg, hipStream_t s) {
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((N * N + 255) / 256)), dim3(256), 0, s, N,
                     chunks, part, G, ldg);
  return hipGetLastError();
}

}  // namespace eda
