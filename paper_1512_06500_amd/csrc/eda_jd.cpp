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

// Column-wise Gram-Schmidt of W (c columns) against blocks U_0 .. U_{blocks-1}
// of c columns each (column j of every block belongs to column j of W):
// g[p c + j] = U_p(:, j)^T W(:, j) is added to acc (host) and W(:, j) -=
// sum_p g[p c + j] U_p(:, j).  Gd, Dd: device scratch of blocks c^2 doubles.
eda_status colwise_gs(eda_handle h, int64_t d, int64_t ldq, const double* U, int64_t blocks,
                      int64_t c, double* W, double* acc, double* Gd, double* Dd) {
  hipStream_t s = h->stream;
  const int64_t m = blocks * c;
  const int64_t chunks = tn_chunks(d, m, c);
  STCHK(ensure(h, h->part, (size_t)chunks * m * c * 8));
  HIPCHK(launch_tn_partial(d, m, c, U, DT::F64, ldq, W, DT::F64, ldq, h->part.d(), chunks, nullptr,
                           s));
  HIPCHK(launch_reduce_partials(chunks, m, c, h->part.d(), 1.0, 0.0, Gd, m, 0.0, nullptr, 0,
                                nullptr, s));
  std::vector<double> G((size_t)m * c), D((size_t)m * c, 0.0);
  HIPCHK(hipMemcpyAsync(G.data(), Gd, G.size() * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int64_t p = 0; p < blocks; ++p)
    for (int64_t j = 0; j < c; ++j) {
      const double g = G[(size_t)(p * c + j) + (size_t)j * m];
      D[(size_t)(p * c + j) * c + j] = -g;
      acc[p * c + j] += g;
    }
  HIPCHK(hipMemcpyAsync(Dd, D.data(), D.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(launch_nn(d, m, c, U, DT::F64, ldq, Dd, c, 1.0, W, DT::F64, ldq, W, DT::F64, ldq, nullptr,
                   s));
  HIPCHK(hipStreamSynchronize(s));  // D is a host temporary
  return EDA_OK;
}

// Column norms of W (c columns) on the host.
eda_status col_norms(eda_handle h, int64_t d, int64_t ldq, const double* W, int64_t c, double* Gd,
                     double* out) {
  hipStream_t s = h->stream;
  const int64_t chunks = tn_chunks(d, c, c);
  STCHK(ensure(h, h->part, (size_t)chunks * c * c * 8));
  HIPCHK(launch_tn_partial(d, c, c, W, DT::F64, ldq, W, DT::F64, ldq, h->part.d(), chunks, nullptr,
                           s));
  HIPCHK(launch_reduce_partials(chunks, c, c, h->part.d(), 1.0, 0.0, Gd, c, 0.0, nullptr, 0,
                                nullptr, s));
  std::vector<double> G((size_t)c * c);
  HIPCHK(hipMemcpyAsync(G.data(), Gd, G.size() * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int64_t j = 0; j < c; ++j) out[j] = std::sqrt(std::max(G[(size_t)j * c + j], 0.0));
  return EDA_OK;
}

// Out(:, j) = sum_q A(:, q) Dm(q, j) with a host matrix Dm (rows x c,
// row-major), copied to the device scratch Dd.
eda_status combine(eda_handle h, int64_t d, int64_t ldq, const double* A, int64_t rows, int64_t c,
                   const std::vector<double>& Dm, double* Dd, double alpha, const double* V,
                   double* Out) {
  hipStream_t s = h->stream;
  HIPCHK(hipMemcpyAsync(Dd, Dm.data(), Dm.size() * 8, hipMemcpyHostToDevice, s));
  HIPCHK(launch_nn(d, rows, c, A, DT::F64, ldq, Dd, c, alpha, V, DT::F64, ldq, Out, DT::F64, ldq,
                   nullptr, s));
  HIPCHK(hipStreamSynchronize(s));
  return EDA_OK;
}

// min || beta e_1 - H y || over y in R^k for the (k+1) x k Hessenberg H
// (column-major, leading dimension ldh) by Givens rotations; columns from
// the first zero subdiagonal entry on are dropped (the Krylov space became
// invariant there and the system is solved).
void gmres_ls(int k, const double* H, int ldh, double beta, double* y) {
  std::vector<double> R((size_t)(k + 1) * k, 0.0);
  for (int l = 0; l < k; ++l)
    for (int p = 0; p <= l + 1; ++p) R[(size_t)l * (k + 1) + p] = H[(size_t)l * ldh + p];
  std::vector<double> g(k + 1, 0.0), cs(k, 1.0), sn(k, 0.0);
  g[0] = beta;
  int kk = k;
  for (int l = 0; l < k; ++l) {
    double* col = R.data() + (size_t)l * (k + 1);
    for (int p = 0; p < l; ++p) {
      const double a = col[p], b2 = col[p + 1];
      col[p] = cs[p] * a + sn[p] * b2;
      col[p + 1] = -sn[p] * a + cs[p] * b2;
    }
    const double a = col[l], b2 = col[l + 1];
    const double r = std::hypot(a, b2);
    if (!(r > 0.0)) {
      kk = l;
      break;
    }
    cs[l] = a / r;
    sn[l] = b2 / r;
    col[l] = r;
    col[l + 1] = 0.0;
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
    for (int q = l + 1; q < kk; ++q) sacc -= R[(size_t)q * (k + 1) + l] * y[q];
    y[l] = sacc / R[(size_t)l * (k + 1) + l];
  }
}

}  // namespace

namespace eda {

eda_status solve_jd(eda_handle h, int32_t t, double tol, const eda_solve_opts& o, double* ritz,
                    double* ritz_log, double* X, int64_t ldx, double* resid, eda_info* info) {
  if (o.krylov_dtype != EDA_F64)
    return fail(h, EDA_ERR_ARG, "the Jacobi-Davidson form runs in float64 (krylov_dtype EDA_F64)");
  const int64_t d = h->d, N = h->N, ldq = h->ldp;
  const int64_t b = o.block > 0 ? o.block : 8;
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
  STCHK(ensure(h, h->af[6], (size_t)(2 * KC * b + 4 * wmax * wmax) * 8));
  double* Bv[2] = {h->af[0].d(), h->af[2].d()};
  double* MBv[2] = {h->af[1].d(), h->af[3].d()};
  double* R = h->af[4].d();
  double* U = h->af[5].d();
  double* W = U + (size_t)ldq * KC;
  double* Gd = h->af[6].d();
  double* Dd = Gd + KC * b;
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
    // U_0 = -r_i / ||r_i||
    {
      std::vector<double> Dm((size_t)kept * c, 0.0);
      for (int64_t j = 0; j < c; ++j) {
        const int64_t i = open[j];
        Dm[(size_t)i * c + j] = res[i] > 0.0 ? -1.0 / res[i] : 0.0;
      }
      STCHK(combine(h, d, ldq, R, kept, c, Dm, Dd, 0.0, nullptr, U));
    }
    std::vector<double> Hh((size_t)c * (kInner + 1) * kInner, 0.0);  // per column (k+1) x k
    std::vector<double> nrm(c), acc((size_t)(kInner + 1) * c);
    std::vector<double> mth((size_t)c * c, 0.0);
    for (int64_t j = 0; j < c; ++j) mth[(size_t)j * c + j] = -theta[open[j]];
    int steps = 0;
    for (int l = 0; l < kInner; ++l) {
      double* Ul = U + (size_t)l * c * ldq;
      // W = (e^{-s} M - theta I) U_l, projected against the kept Ritz vectors
      STCHK(expop(h, true, 0, N, h->CM.d(), N, h->alphaB, c, Ul, DT::F64, ldq, W, DT::F64, ldq));
      ops += c;
      STCHK(combine(h, d, ldq, Ul, c, c, mth, Dd, 1.0, W, W));
      STCHK(cgs_pass(h, d, kept, Y, DT::F64, ldq, W, ldq, c, nullptr, 0, 0.0, nullptr));
      // Arnoldi coefficients against U_0 .. U_l (classical Gram-Schmidt, twice)
      std::fill(acc.begin(), acc.end(), 0.0);
      STCHK(colwise_gs(h, d, ldq, U, l + 1, c, W, acc.data(), Gd, Dd));
      STCHK(colwise_gs(h, d, ldq, U, l + 1, c, W, acc.data(), Gd, Dd));
      STCHK(col_norms(h, d, ldq, W, c, Gd, nrm.data()));
      std::vector<double> sc((size_t)c * c, 0.0);
      for (int64_t j = 0; j < c; ++j) {
        double* Hj = Hh.data() + (size_t)j * (kInner + 1) * kInner;
        for (int p = 0; p <= l; ++p) Hj[(size_t)l * (kInner + 1) + p] = acc[(size_t)p * c + j];
        // a column whose Krylov space became invariant stops (zero next vector)
        const bool stop = !(nrm[j] > 1e-14 * std::fabs(theta[0]));
        Hj[(size_t)l * (kInner + 1) + l + 1] = stop ? 0.0 : nrm[j];
        sc[(size_t)j * c + j] = stop ? 0.0 : 1.0 / nrm[j];
      }
      STCHK(combine(h, d, ldq, W, c, c, sc, Dd, 0.0, nullptr, U + (size_t)(l + 1) * c * ldq));
      steps = l + 1;
    }
    // z_j = sum_l y_j[l] U_l(:, j), y_j from the small least-squares problems
    // (right-hand side ||-r_j|| e_1 in the basis U_0 = -r_j / ||r_j||)
    {
      std::vector<double> Dm((size_t)steps * c * c, 0.0), y(kInner);
      for (int64_t j = 0; j < c; ++j) {
        gmres_ls(steps, Hh.data() + (size_t)j * (kInner + 1) * kInner, kInner + 1, res[open[j]],
                 y.data());
        for (int l = 0; l < steps; ++l) Dm[(size_t)(l * c + j) * c + j] = y[l];
      }
      // the corrections go to the search-space slots after the kept vectors
      STCHK(combine(h, d, ldq, U, steps * c, c, Dm, Dd, 0.0, nullptr, Y + (size_t)kept * ldq));
    }
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
    info->t_prepare_ms = h->t_prepare_ms;
    info->t_krylov_ms = kms;
    info->shift_s = h->shiftB;
  }
  if (range_err) return fail(h, EDA_ERR_RANGE, "a Ritz value underflowed after the shift");
  if (!converged)
    return fail(h, EDA_ERR_NOCONV, "Jacobi-Davidson: max_iter reached before convergence");
  return EDA_OK;
}

}  // namespace eda
