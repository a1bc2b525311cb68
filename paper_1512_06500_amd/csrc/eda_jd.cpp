// libeda host library: eda_solve by block Jacobi-Davidson.
//
// An eigensolver of the Jacobi-Davidson family, which the paper's closing
// section names as a further way to reach the dominant eigenpairs of the
// exponential pencil, here on the symmetric e^{-s} M of eq. (3.15) with the
// same streaming products (Theorem 3.1) as block Lanczos.  Each outer step
//   1. takes the Rayleigh-Ritz pairs (theta_i, y_i) of the search space and
//      the explicit residuals r_i = e^{-s} M y_i - theta_i y_i;
//   2. for up to b unconverged pairs, solves the correction equation
//        (I - Y Y^T)(e^{-s} M - theta_i I)(I - Y Y^T) z_i = -r_i,  z_i _|_ Y,
//      approximately by kInner steps of GMRES, all columns in lockstep (one
//      block product with e^{-s} M per step; Y = the kept Ritz vectors);
//   3. restarts the search space to the t + b leading Ritz vectors plus the
//      orthonormalised corrections.
// Float64 throughout, on the float64 operator; the back-transform and the
// orthonormalisation of the result are those of the Lanczos form.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "host_internal.h"

using namespace eda;

namespace {

constexpr int kInner = 4;  // GMRES steps per correction

// Gram block X^T Y (rows x c, column-major, leading dimension rows) into G.
eda_status gram_block(eda_handle h, int64_t d, int64_t ldq, const double* X, int64_t rows,
                      const double* Y, int64_t c, double* G) {
  const int64_t chunks = tn_chunks(d, rows, c);
  STCHK(ensure(h, h->part, (size_t)chunks * rows * c * 8));
  HIPCHK(launch_tn_partial(d, rows, c, X, DT::F64, ldq, Y, DT::F64, ldq, h->part.d(), chunks,
                           nullptr, h->stream));
  HIPCHK(launch_reduce_partials(chunks, rows, c, h->part.d(), 1.0, 0.0, G, rows, 0.0, nullptr, 0,
                                nullptr, h->stream));
  return EDA_OK;
}

}  // namespace

namespace eda {

eda_status solve_jd(eda_handle h, int32_t t, double tol, const eda_solve_opts& o, double* ritz,
                    double* ritz_log, double* X, int64_t ldx, double* resid, eda_info* info) {
  if (o.krylov_dtype != EDA_F64)
    return fail(h, EDA_ERR_ARG, "the Jacobi-Davidson form runs in float64 (krylov_dtype EDA_F64)");
  const int64_t d = h->d, N = h->N, ldq = h->ldp;
  const int64_t b = o.block > 0 ? o.block : 8;
  if (b > 8) return fail(h, EDA_ERR_ARG, "the Jacobi-Davidson form takes block widths in [1, 8]");
  const int64_t nk = t + b;                   // Ritz vectors kept at every restart
  const int64_t wmax = nk + b;                // search space columns
  if (wmax > d) return fail(h, EDA_ERR_ARG, "Jacobi-Davidson needs t + 2b <= d");
  const int64_t max_iter = o.max_iter > 0 ? o.max_iter : 1000;
  hipStream_t s = h->stream;
  const int64_t mm = wmax;
  const int64_t KC = (int64_t)(kInner + 1) * b;  // inner basis columns

  // buffers: search space and its image (two of each), residuals, inner
  // basis, small device scratch
  STCHK(ensure(h, h->af[0], (size_t)ldq * wmax * 8));
  STCHK(ensure(h, h->af[1], (size_t)ldq * wmax * 8));
  STCHK(ensure(h, h->af[2], (size_t)ldq * wmax * 8));
  STCHK(ensure(h, h->af[3], (size_t)ldq * wmax * 8));
  STCHK(ensure(h, h->af[4], (size_t)ldq * nk * 8));
  STCHK(ensure(h, h->af[5], (size_t)ldq * (KC + b) * 8));
  // device scratch: Gram blocks, update and scale matrices, the Hessenberg
  // matrices of the c columns, and the per-step inputs (U_0 mixing, -theta,
  // beta) uploaded from pinned memory once per outer step
  const int64_t nstage = nk * b + b * b + b;
  STCHK(ensure(h, h->af[6], (size_t)(2 * KC * b + b * b + b * (kInner + 1) * kInner + nstage) * 8));
  double* Bv[2] = {h->af[0].d(), h->af[2].d()};
  double* MBv[2] = {h->af[1].d(), h->af[3].d()};
  double* R = h->af[4].d();
  double* U = h->af[5].d();
  double* W = U + (size_t)ldq * KC;
  double* Gd = h->af[6].d();
  double* Dd = Gd + KC * b;
  double* Sg = Dd + KC * b;
  double* Hd = Sg + b * b;
  double* stage_d = Hd + b * (kInner + 1) * kInner;
  double* stage_h = nullptr;
  if (hipHostMalloc((void**)&stage_h, (size_t)nstage * 8, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, EDA_ERR_NOMEM, "pinned staging of %lld doubles failed", (long long)nstage);
  }
  struct PinGuard {
    double* p;
    ~PinGuard() { (void)hipHostFree(p); }
  } pin_guard{stage_h};
  STCHK(ensure(h, h->T, (size_t)mm * mm * 8));
  STCHK(ensure(h, h->wT, (size_t)mm * 8));
  STCHK(ensure(h, h->S, (size_t)mm * mm * 8));
  STCHK(ensure(h, h->Sd, (size_t)mm * nk * 8));
  STCHK(ensure(h, h->dtheta, (size_t)(nk + 8) * 8));
  STCHK(ensure(h, h->dres, (size_t)(nk + 8) * 8));
  STCHK(ensure(h, h->syev_work, syev_work_bytes(mm)));
  STCHK(ensure(h, h->flags, 64));
  STCHK(ensure(h, h->mask, 128 * sizeof(int)));
  STCHK(ensure(h, h->Yb, (size_t)ldq * std::max<int64_t>(t, b) * 8));
  STCHK(ensure(h, h->Gs, (size_t)wmax * wmax * 8));
  STCHK(ensure(h, h->Rinv, (size_t)wmax * wmax * 8));
  STCHK(ensure(h, h->R1, (size_t)b * b * 8));
  STCHK(ensure(h, h->hz, (size_t)wmax * wmax * 8));
  STCHK(ensure(h, h->Ysm, (size_t)N * wmax * 8));
  STCHK(ensure(h, h->Zsm, (size_t)N * wmax * 8));
  HIPCHK(launch_fill_i32(16, 0, h->flags.i(), s));
  h->op_used = 0;

  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));

  // initial search space: the start block (or Gaussian columns) and
  // Gaussian columns up to t + b, orthonormalised; its image
  int cur = 0;
  int64_t w = nk;
  double* B = Bv[cur];
  HIPCHK(launch_randn(d, w, o.seed, B, ldq, s));
  if (o.start_block != nullptr)
    HIPCHK(launch_copy2d(d, b, o.start_block, DT::F64, o.ld_start, B, DT::F64, ldq, s));
  // (Cholesky QR twice, through the other buffer: the product is not in place)
  STCHK(cholqr_pass(h, d, w, B, DT::F64, ldq, Bv[1], ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                    nullptr, nullptr));
  STCHK(cholqr_pass(h, d, w, Bv[1], DT::F64, ldq, B, ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                    nullptr, nullptr));
  STCHK(expop(h, true, 0, N, h->CM.d(), N, h->alphaB, w, B, DT::F64, ldq, MBv[cur], DT::F64, ldq));
  int64_t ops = w;

  std::vector<double> theta(nk), res(nk);
  bool converged = false, floor_limited = false;
  int64_t iters = 0;
  double* Y = nullptr;
  double* MY = nullptr;
  while (true) {
    // 1. Rayleigh-Ritz: the nk leading pairs to the other buffer
    const int64_t kept = std::min<int64_t>(nk, w);
    double* B2 = Bv[1 - cur];
    double* MB2 = MBv[1 - cur];
    STCHK(rr_block(h, d, ldq, w, kept, mm, Bv[cur], MBv[cur], B2, MB2));
    HIPCHK(launch_ritz_residual(d, kept, MB2, ldq, B2, ldq, h->dtheta.d(), R, ldq, h->dres.d(), s));
    HIPCHK(hipMemcpyAsync(theta.data(), h->dtheta.d(), kept * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(res.data(), h->dres.d(), kept * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    Y = B2;
    MY = MB2;
    cur = 1 - cur;
    // stopping test of the Lanczos form (per-pair floors 10 u theta_1 / theta_i)
    bool ok = true;
    floor_limited = false;
    std::vector<int64_t> open;
    for (int64_t i = 0; i < t; ++i) {
      const double thi = theta[i];
      bool pass = thi > 0.0;
      if (pass) {
        const double floor_i = 10.0 * kU64 * theta[0] / thi;
        if (floor_i > tol) floor_limited = true;
        const double r = (o.resmode == EDA_RES_REL_THETA) ? res[i] / thi : res[i] / theta[0];
        pass = r <= std::max(tol, floor_i);
      }
      if (!pass) {
        ok = false;
        open.push_back(i);
      }
    }
    if (ok) {
      converged = true;
      break;
    }
    if (iters >= max_iter) break;
    ++iters;
    // 2. corrections for the first c open pairs
    const int64_t c = std::min<int64_t>(b, (int64_t)open.size());
    // per-step inputs: U_0 = -r_i / ||r_i|| as a mixing of the residuals,
    // -theta_i on a diagonal, beta_i = ||r_i||
    {
      double* mix = stage_h;
      double* mth = stage_h + kept * c;
      double* beta = mth + c * c;
      std::fill(stage_h, stage_h + kept * c + c * c + c, 0.0);
      for (int64_t j = 0; j < c; ++j) {
        const int64_t i = open[j];
        mix[i * c + j] = res[i] > 0.0 ? -1.0 / res[i] : 0.0;
        mth[j * c + j] = -theta[i];
        beta[j] = res[i];
      }
      HIPCHK(hipMemcpyAsync(stage_d, stage_h, (size_t)(kept * c + c * c + c) * 8,
                            hipMemcpyHostToDevice, s));
    }
    const double* mix_d = stage_d;
    const double* mth_d = stage_d + kept * c;
    const double* beta_d = mth_d + c * c;
    HIPCHK(launch_nn(d, kept, c, R, DT::F64, ldq, mix_d, c, 0.0, nullptr, DT::F64, ldq, U, DT::F64,
                     ldq, nullptr, s));
    HIPCHK(launch_fill(c * (kInner + 1) * kInner, 0.0, Hd, s));
    const double tiny = 1e-14 * std::fabs(theta[0]);
    for (int l = 0; l < kInner; ++l) {
      double* Ul = U + (size_t)l * c * ldq;
      // W = (e^{-s} M - theta I) U_l, projected against the kept Ritz vectors
      STCHK(expop(h, true, 0, N, h->CM.d(), N, h->alphaB, c, Ul, DT::F64, ldq, W, DT::F64, ldq));
      ops += c;
      HIPCHK(launch_nn(d, c, c, Ul, DT::F64, ldq, mth_d, c, 1.0, W, DT::F64, ldq, W, DT::F64, ldq,
                       nullptr, s));
      STCHK(cgs_pass(h, d, kept, Y, DT::F64, ldq, W, ldq, c, nullptr, 0, 0.0, nullptr));
      // Arnoldi coefficients against U_0 .. U_l (column-wise classical
      // Gram-Schmidt, twice), the norm and the next basis block
      for (int pass = 0; pass < 2; ++pass) {
        STCHK(gram_block(h, d, ldq, U, (l + 1) * c, W, c, Gd));
        HIPCHK(launch_jd_gs_coeffs(l + 1, (int)c, kInner, l, Gd, Dd, Hd, s));
        HIPCHK(launch_nn(d, (l + 1) * c, c, U, DT::F64, ldq, Dd, c, 1.0, W, DT::F64, ldq, W,
                         DT::F64, ldq, nullptr, s));
      }
      STCHK(gram_block(h, d, ldq, W, c, W, c, Gd));
      HIPCHK(launch_jd_norms((int)c, kInner, l, Gd, tiny, Sg, Hd, s));
      HIPCHK(launch_nn(d, c, c, W, DT::F64, ldq, Sg, c, 0.0, nullptr, DT::F64, ldq,
                       U + (size_t)(l + 1) * c * ldq, DT::F64, ldq, nullptr, s));
    }
    // z_j = sum_l y_j[l] U_l(:, j), y_j from the small least-squares problems
    // (right-hand side ||r_j|| e_1 in the basis U_0 = -r_j / ||r_j||); the
    // corrections go to the search-space slots after the kept vectors
    HIPCHK(launch_jd_gmres_ls((int)c, kInner, Hd, beta_d, Dd, s));
    HIPCHK(launch_nn(d, kInner * c, c, U, DT::F64, ldq, Dd, c, 0.0, nullptr, DT::F64, ldq,
                     Y + (size_t)kept * ldq, DT::F64, ldq, nullptr, s));
    // 3. orthonormalise the corrections against the kept Ritz vectors and
    // among themselves (rank revealing: a correction already inside the
    // space is replaced by a random direction), then their image
    double* Z = Y + (size_t)kept * ldq;
    STCHK(cgs_pass(h, d, kept, Y, DT::F64, ldq, Z, ldq, c, nullptr, 0, 0.0, nullptr));
    STCHK(cgs_pass(h, d, kept, Y, DT::F64, ldq, Z, ldq, c, nullptr, 0, 0.0, nullptr));
    {
      const int64_t chunks = tn_chunks(d, c, c);
      STCHK(ensure(h, h->part, (size_t)chunks * c * c * 8));
      HIPCHK(launch_tn_partial(d, c, c, Z, DT::F64, ldq, Z, DT::F64, ldq, h->part.d(), chunks,
                               nullptr, s));
      HIPCHK(launch_pchol(c, h->Gs.d(), c, nullptr, 0, 0, 1e-10, 1e-4, true, h->Rinv.d(), c,
                          h->R1.d(), c, h->mask.i(), nullptr, s, h->part.d(), chunks));
      HIPCHK(launch_nn(d, c, c, Z, DT::F64, ldq, h->Rinv.d(), c, 0.0, nullptr, DT::F64, ldq, W,
                       DT::F64, ldq, nullptr, s, false, nullptr, nullptr, h->mask.i(),
                       0x3d1e0000ull + (uint64_t)iters));
    }
    STCHK(cgs_pass(h, d, kept, Y, DT::F64, ldq, W, ldq, c, nullptr, 0, 0.0, nullptr));
    STCHK(cgs_pass(h, d, kept, Y, DT::F64, ldq, W, ldq, c, nullptr, 0, 0.0, nullptr));
    STCHK(cholqr_pass(h, d, c, W, DT::F64, ldq, Z, ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                      nullptr, nullptr));
    STCHK(cholqr_pass(h, d, c, Z, DT::F64, ldq, Z, ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                      nullptr, nullptr));
    STCHK(expop(h, true, 0, N, h->CM.d(), N, h->alphaB, c, Z, DT::F64, ldq,
                MY + (size_t)kept * ldq, DT::F64, ldq));
    ops += c;
    w = kept + c;
  }
  HIPCHK(hipEventRecord(e1, s));
  // back-transform x = exp(-S_W/2) y of the t leading Ritz vectors,
  // orthonormalised in decreasing-lambda order, signs fixed
  STCHK(back_transform(h, t, Y, ldq, X, ldx, ldq));
  int fl[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(fl, h->flags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  float kms = 0.f;
  HIPCHK(hipEventElapsedTime(&kms, e0, e1));
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
    resid[i] = (o.resmode == EDA_RES_REL_THETA) ? res[i] / th : res[i] / theta[0];
  }
  if (info != nullptr) {
    std::memset(info, 0, sizeof(*info));
    info->iters = (int32_t)iters;
    info->flags = (floor_limited ? EDA_WARN_FLOOR : 0) | ((fl[0] | fl[1]) ? EDA_WARN_REPAIRED : 0);
    info->ops = ops;
    info->bytes_moved = (double)ops / b * (2.0 * d * N * 8.0 + 3.0 * d * b * 8.0);
    info->t_prepare_ms = prepare_time_ms(h);
    info->t_krylov_ms = kms;
    info->shift_s = h->shiftB;
  }
  if (range_err) return fail(h, EDA_ERR_RANGE, "a Ritz value underflowed after the shift");
  if (!converged)
    return fail(h, EDA_ERR_NOCONV, "Jacobi-Davidson: max_iter reached before convergence");
  return EDA_OK;
}

}  // namespace eda
