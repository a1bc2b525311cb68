// Small kernels of the block Jacobi-Davidson inner solve (eda_jd.cpp): the
// column-wise Gram-Schmidt coefficients, the column norms and the GMRES
// least-squares problems of the c columns in lockstep, kept on the device so
// that the inner steps need no host round trip.  Column j of the lockstep
// owns the upper Hessenberg matrix H_j ((k + 1) x k, column-major, leading
// dimension k + 1) at H + j (k + 1) k.
#include <hip/hip_runtime.h>

#include "common.h"

namespace eda {

namespace {

// G (blocks c x c, column-major, ld blocks c) = U^T W for blocks of c
// columns: coefficient g = G(p c + j, j) goes to H_j(p, l) (added) and to
// D(p c + j, j) = -g of the row-major update matrix (all other entries 0).
__global__ __launch_bounds__(256) void jd_gs_coeffs_kernel(int blocks, int c, int k, int l,
                                                           const double* __restrict__ G,
                                                           double* __restrict__ D,
                                                           double* __restrict__ H) {
  const int m = blocks * c;
  const int r = blockIdx.x * 256 + threadIdx.x;  // row p c + j of D
  if (r >= m) return;
  const int p = r / c, j = r - p * c;
  const double g = G[r + (int64_t)j * m];
  for (int q = 0; q < c; ++q) D[(int64_t)r * c + q] = (q == j) ? -g : 0.0;
  H[(int64_t)j * (k + 1) * k + (int64_t)l * (k + 1) + p] += g;
}

// G = W^T W (c x c): H_j(l + 1, l) = ||W(:, j)|| and S = diag(1 / norm),
// row-major; a column whose norm is at most `tiny` stops (zero entry, zero
// scale: its next basis vector is zero).
__global__ __launch_bounds__(64) void jd_norms_kernel(int c, int k, int l,
                                                      const double* __restrict__ G, double tiny,
                                                      double* __restrict__ S,
                                                      double* __restrict__ H) {
  const int j = threadIdx.x;
  if (j >= c) return;
  const double nrm = sqrt(fmax(G[j + (int64_t)j * c], 0.0));
  const bool stop = !(nrm > tiny);
  H[(int64_t)j * (k + 1) * k + (int64_t)l * (k + 1) + l + 1] = stop ? 0.0 : nrm;
  for (int q = 0; q < c; ++q) S[(int64_t)j * c + q] = (q == j && !stop) ? 1.0 / nrm : 0.0;
}

// min || beta_j e_1 - H_j y || by Givens rotations, one thread per column;
// columns from the first zero subdiagonal entry on are dropped.  The
// solution goes to column j of Y (row-major, (k c) x c: Y(l c + j, j) = y_l,
// zero elsewhere in column j).
constexpr int kJdMaxK = 8;
__global__ __launch_bounds__(64) void jd_gmres_ls_kernel(int c, int k, const double* __restrict__ H,
                                                         const double* __restrict__ beta,
                                                         double* __restrict__ Y) {
  const int j = threadIdx.x;
  if (j >= c) return;
  const double* Hj = H + (int64_t)j * (k + 1) * k;
  double R[kJdMaxK + 1][kJdMaxK];
  double g[kJdMaxK + 1], cs[kJdMaxK], sn[kJdMaxK], y[kJdMaxK];
  for (int l = 0; l < k; ++l)
    for (int p = 0; p <= k; ++p) R[p][l] = (p <= l + 1) ? Hj[l * (k + 1) + p] : 0.0;
  for (int p = 0; p <= k; ++p) g[p] = 0.0;
  g[0] = beta[j];
  int kk = k;
  for (int l = 0; l < k; ++l) {
    for (int p = 0; p < l; ++p) {
      const double a = R[p][l], b2 = R[p + 1][l];
      R[p][l] = cs[p] * a + sn[p] * b2;
      R[p + 1][l] = -sn[p] * a + cs[p] * b2;
    }
    const double a = R[l][l], b2 = R[l + 1][l];
    const double r = hypot(a, b2);
    if (!(r > 0.0)) {
      kk = l;
      break;
    }
    cs[l] = a / r;
    sn[l] = b2 / r;
    R[l][l] = r;
    R[l + 1][l] = 0.0;
    const double g0 = g[l];
    g[l] = cs[l] * g0;
    g[l + 1] = -sn[l] * g0;
    if (b2 == 0.0) {
      kk = l + 1;
      break;
    }
  }
  for (int l = 0; l < k; ++l) y[l] = 0.0;
  for (int l = kk - 1; l >= 0; --l) {
    double sacc = g[l];
    for (int q = l + 1; q < kk; ++q) sacc -= R[l][q] * y[q];
    y[l] = sacc / R[l][l];
  }
  for (int l = 0; l < k; ++l)
    for (int q = 0; q < c; ++q) Y[(int64_t)(l * c + q) * c + j] = (q == j) ? y[l] : 0.0;
}

}  // namespace

hipError_t launch_jd_gs_coeffs(int blocks, int c, int k, int l, const double* G, double* D,
                               double* H, hipStream_t s) {
  if (blocks < 1 || c < 1 || c > 64 || k < 1 || k > kJdMaxK || l < 0 || l >= k || blocks > k)
    return hipErrorInvalidValue;
  const int m = blocks * c;
  hipLaunchKernelGGL(jd_gs_coeffs_kernel, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s,
                     blocks, c, k, l, G, D, H);
  return hipGetLastError();
}

hipError_t launch_jd_norms(int c, int k, int l, const double* G, double tiny, double* S,
                           double* H, hipStream_t s) {
  if (c < 1 || c > 64 || k < 1 || k > kJdMaxK || l < 0 || l >= k) return hipErrorInvalidValue;
  hipLaunchKernelGGL(jd_norms_kernel, dim3(1), dim3(64), 0, s, c, k, l, G, tiny, S, H);
  return hipGetLastError();
}

hipError_t launch_jd_gmres_ls(int c, int k, const double* H, const double* beta, double* Y,
                              hipStream_t s) {
  if (c < 1 || c > 64 || k < 1 || k > kJdMaxK) return hipErrorInvalidValue;
  hipLaunchKernelGGL(jd_gmres_ls_kernel, dim3(1), dim3(64), 0, s, c, k, H, beta, Y);
  return hipGetLastError();
}

}  // namespace eda
