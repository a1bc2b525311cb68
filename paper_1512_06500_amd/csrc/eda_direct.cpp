// Reduced direct solve: the whole pencil (1.7) on the GPU without a Krylov
// iteration.  Both exponentials are the identity plus a low-rank term in
// span P, P = [H_W H_B] (Theorem 3.1), so the operator iterated by the
// Lanczos solver,
//   e^{-s} M = alpha I + P C_M P^T       (alpha = e^{-s}, core C_M of the composite product),
// has the eigenvalue alpha on the orthogonal complement of span P and on
// span P the eigenvalues of an r x r matrix, r = rank P.  With the Gram
// matrix G = P^T P = V diag(w) V^T and F = V_r diag(sqrt(w_r)) (the r
// leading eigenpairs), U = P V_r diag(w_r)^{-1/2} is an orthonormal basis of
// span P with U^T P = F^T, so
//   U^T (e^{-s} M) U = alpha I + F^T C_M F = K   (r x r, symmetric).
// The t leading eigenpairs (theta, z) of K give the Ritz pairs of M exactly:
// lambda = e^{s} theta and y = U z = P (V_r diag(w_r)^{-1/2} z), followed by
// the back-transform x = exp(-S_W/2) y of eq. (3.14) and the
// orthonormalisation of Algorithm 3.  Costs two dense eigensolves (N and r)
// and small GEMMs after the Gram matrix of the preparation; the residuals
// are measured with one more product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "host_internal.h"

using namespace eda;

namespace {

enum { kGw = 0, kGZ, kF, kT, kK, kKw, kKZ, kSd, kW, kY };

}  // namespace

extern "C" eda_status eda_solve_direct(eda_handle h, int32_t t, double* ritz, double* ritz_log,
                                       double* X, int64_t ldx, double* resid, eda_info* info) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (!h->prepared) return fail(h, EDA_ERR_STATE, "eda_prepare has not succeeded");
  const int64_t d = h->d, N = h->N;
  if (t < 1 || t >= d || t > N) return fail(h, EDA_ERR_ARG, "need 1 <= t < d and t <= n + k");
  if (t > 128) return fail(h, EDA_ERR_ARG, "t > 128 is not supported");
  if (N > 2048) return fail(h, EDA_ERR_ARG, "n + k = %lld exceeds 2048 (dense eigensolve)",
                            (long long)N);
  if (ritz == nullptr || ritz_log == nullptr || X == nullptr || resid == nullptr)
    return fail(h, EDA_ERR_ARG, "null output pointer");
  if (ldx < d) return fail(h, EDA_ERR_ARG, "ldx must be >= d");
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, X, "X"));
  hipStream_t s = h->stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));

  // leading eigenpairs of the Gram matrix, rank by the float64 floor.  The
  // class-centred columns of H_W sum to zero within each class and the
  // weighted columns of H_B sum to zero, so rank P <= n - 1: only the n - 1
  // leading pairs are computed (the null space is never resolved).
  Buf* B = h->dir;
  const int64_t nv = std::min<int64_t>(N, h->n - 1);
  STCHK(ensure(h, B[kGw], (size_t)N * 8));
  STCHK(ensure(h, B[kGZ], (size_t)N * N * 8));
  STCHK(ensure(h, h->syev_work, syev_work_bytes(N)));
  HIPCHK(launch_syev(1, N, nullptr, h->G.d(), N, 0, B[kGw].d(), 0, B[kGZ].d(), N, 0, nv,
                     h->syev_work.d(), s));
  std::vector<double> gw(N);
  HIPCHK(hipMemcpyAsync(gw.data(), B[kGw].d(), N * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double wmax = gw[N - 1];
  const double thr = (double)N * 0x1.0p-52 * wmax;
  int64_t r = 0;
  for (int64_t i = 0; i < N; ++i) r += (gw[i] > thr);
  if (!(wmax > 0.0) || r < t) return fail(h, EDA_ERR_ARG, "t=%d exceeds rank P = %lld", t, (long long)r);
  const double* Vr = B[kGZ].d() + (N - r) * N;
  const double* wr = B[kGw].d() + (N - r);

  // K = alpha I + F^T C_M F,  F = V_r diag(sqrt(w_r))
  STCHK(ensure(h, B[kF], (size_t)N * r * 8));
  STCHK(ensure(h, B[kT], (size_t)N * r * 8));
  STCHK(ensure(h, B[kK], (size_t)r * r * 8));
  STCHK(ensure(h, B[kKw], (size_t)r * 8));
  HIPCHK(launch_scale_cols(N, r, Vr, N, wr, +1, B[kF].d(), N, s));
  HIPCHK(launch_gemm(false, false, N, r, N, 1.0, h->CM.d(), N, nullptr, B[kF].d(), N, 0.0,
                     B[kT].d(), N, s));
  HIPCHK(launch_fill(r * r, 0.0, B[kK].d(), s));
  HIPCHK(launch_fill(r, h->alphaB, B[kKw].d(), s));
  HIPCHK(launch_set_diag(r, B[kKw].d(), B[kK].d(), r, s));
  HIPCHK(launch_gemm(true, false, r, r, N, 1.0, B[kF].d(), N, nullptr, B[kT].d(), N, 1.0,
                     B[kK].d(), r, s));

  // the t leading eigenpairs of K (descending), z as rows of Sd
  STCHK(ensure(h, B[kKZ], (size_t)r * r * 8));
  STCHK(ensure(h, B[kSd], (size_t)r * t * 8));
  STCHK(ensure(h, h->dtheta, (size_t)t * 8));
  HIPCHK(launch_syev(1, r, nullptr, B[kK].d(), r, 0, B[kKw].d(), 0, B[kKZ].d(), r, 0, t,
                     h->syev_work.d(), s));
  HIPCHK(launch_desc_values(t, B[kKw].d(), r, h->dtheta.d(), s));
  HIPCHK(launch_gather_desc(r, t, B[kKZ].d(), r, B[kSd].d(), t, s));

  // Y = P W,  W = V_r diag(w_r)^{-1/2} Z  (N x t, row-major)
  const int64_t ldy = h->ldp;
  STCHK(ensure(h, B[kW], (size_t)N * t * 8));
  STCHK(ensure(h, B[kY], (size_t)ldy * 2 * t * 8));
  double* Y = B[kY].d();
  double* MY = Y + (size_t)ldy * t;
  HIPCHK(launch_scale_cols(N, r, Vr, N, wr, -1, B[kF].d(), N, s));
  HIPCHK(launch_nn(N, r, t, B[kF].d(), DT::F64, N, B[kSd].d(), t, 0.0, nullptr, DT::F64, 0,
                   B[kW].d(), DT::F64, t, nullptr, s, true));
  const bool use64 = h->storage != EDA_F64;
  const void* P = use64 ? h->P64.p : h->P.p;
  HIPCHK(launch_nn(d, N, t, P, DT::F64, h->ldp, B[kW].d(), t, 0.0, nullptr, DT::F64, 0, Y, DT::F64,
                   ldy, nullptr, s));

  // residuals ||e^{-s} M y - theta y|| with the float64 operator
  STCHK(expop(h, true, 0, N, h->CM.d(), N, h->alphaB, t, Y, DT::F64, ldy, MY, DT::F64, ldy));
  STCHK(ensure(h, h->dres, (size_t)t * 8));
  STCHK(ensure(h, h->refine, (size_t)ldy * t * 8));
  HIPCHK(launch_ritz_residual(d, t, MY, ldy, Y, ldy, h->dtheta.d(), h->refine.d(), ldy,
                              h->dres.d(), s));
  std::vector<double> theta(t), res(t);
  HIPCHK(hipMemcpyAsync(theta.data(), h->dtheta.d(), t * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(res.data(), h->dres.d(), t * 8, hipMemcpyDeviceToHost, s));

  // x = exp(-S_W/2) y, orthonormalised in decreasing-lambda order
  STCHK(back_transform(h, t, Y, ldy, X, ldx, ldy));
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);

  bool range_err = false;
  for (int64_t i = 0; i < t; ++i) {
    const double th = theta[i];
    if (!(th > 0.0)) {
      range_err = true;
      ritz_log[i] = -INFINITY;
      ritz[i] = 0.0;
    } else {
      ritz_log[i] = h->shiftB + std::log(th);
      ritz[i] = std::exp(ritz_log[i]);
    }
    resid[i] = res[i] / th;
  }
  if (info != nullptr) {
    std::memset(info, 0, sizeof(*info));
    info->flags = (t > h->k - 1) ? EDA_WARN_DEGENERATE : 0;
    info->ops = 2 * t;
    info->bytes_moved = 2.0 * (2.0 * d * N * 8.0 + 3.0 * d * t * 8.0);
    info->t_prepare_ms = prepare_time_ms(h);
    info->t_krylov_ms = ms;
    info->shift_s = h->shiftB;
  }
  if (range_err) return fail(h, EDA_ERR_RANGE, "a Ritz value is not positive");
  return EDA_OK;
}
