// libeda host library: eda_solve in the Arnoldi form (eq. 3.1).
//
// The t leading eigenpairs of A = exp(-S_W) exp(S_B), whose eigenvectors are
// those of the pencil (1.7) itself, so x comes out directly instead of
// through the back-transform x = exp(-S_W/2) y of the Lanczos form.
//
// A is self-adjoint in the inner product <u, v>_W = u^T exp(S_W) v, so the
// Krylov process used here is block Lanczos in that inner product: the same
// Krylov space as the paper's Arnoldi process on A, with a symmetric
// projected matrix T = V^T exp(S_W) (e^{-s} A) V and real Ritz values.  One
// block step, with BV = exp(S_W) V kept beside the basis V:
//   W = e^{-s} A V_j                 one product with the core C_A (eq. 3.2)
//   h = BV^T W,  W -= V h            (twice; h = <V, W>_W)
//   Z = exp(S_W) W                   one product with the H_W columns of P
//   W = V_{j+1} R,  R^T R = W^T Z   (Cholesky QR in <,>_W, then once more)
//   BV_{j+1} = Z R^{-1}
// exp(S_W) W is formed by a product rather than carried along as Z - BV h:
// that recurrence multiplies the rounding error of BV by ||h|| / ||R|| every
// step, which is large once the Ritz pairs start to converge.  Thick restart
// keeps the leading Ritz vectors (V S and BV S) and the next block.  The
// Ritz vectors x = V s are exp(S_W)-orthonormal; the residual reported is
// the exp(-S_W) norm of r = e^{-s} exp(S_B) x - theta exp(S_W) x, that is
// sqrt(D^T exp(S_W) D) with D = e^{-s} A x - theta x, which equals the
// residual of the Lanczos form for y = exp(S_W/2) x.  The vectors are
// returned orthonormalised in decreasing-lambda order (Algorithm 3, step 6).
//
// The form is float64 throughout.  The inner product has condition number
// e^{lambda_max(S_W)}, so it is refused when ||S_W|| > 12 ln 10.  The basis
// is kept below the dimension of the Krylov space's invariant hull
// (rank P + b <= n - 1 + b), and a block that still loses rank ends the solve
// with EDA_ERR_NOCONV.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host_internal.h"

using namespace eda;

namespace {

enum { kV0 = 0, kV1, kB0, kB1, kH0, kH1, kW, kZ, kG, kGp };

struct AForm {
  eda_handle h;
  int64_t d, n, k, b, t, ldq, ldh, mmax, mm, kk;
  int cur = 0;
  double* V(int q) const { return h->af[q ? kV1 : kV0].d(); }
  double* BV(int q) const { return h->af[q ? kB1 : kB0].d(); }
  double* H(int q) const { return h->af[q ? kH1 : kH0].d(); }
};

// Out = e^{-s} A X = e^{-s} X + P C_A P^T X
eda_status apply_a(const AForm& F, int64_t cols, const double* X, int64_t ldx, double* Out,
                   int64_t ldo) {
  eda_handle h = F.h;
  return expop(h, true, 0, h->N, h->CA.d(), h->N, h->alphaB, cols, X, DT::F64, ldx, Out, DT::F64,
               ldo);
}

// Out = exp(S_W) X: the first n columns of P, core phi_1(G_WW)
eda_status apply_w(const AForm& F, int64_t cols, const double* X, int64_t ldx, double* Out,
                   int64_t ldo) {
  eda_handle h = F.h;
  return expop(h, true, 0, F.n, h->af[kGp].d(), F.n, 1.0, cols, X, DT::F64, ldx, Out, DT::F64,
               ldo);
}

// One Gram-Schmidt pass in <,>_W against the first m basis columns:
// c = BV^T W (= <V, W>_W; into Hcol, accumulated when beta = 1, skipped when
// Hcol is null), W -= V c, and U -= BV c when U is given.
eda_status project(const AForm& F, int64_t m, double* W, double* U, double* Hcol, double beta,
                   const int* gate) {
  eda_handle h = F.h;
  hipStream_t s = h->stream;
  const int64_t chunks = tn_chunks(F.d, m, F.b);
  STCHK(ensure(h, h->part, (size_t)chunks * m * F.b * 8));
  HIPCHK(launch_tn_partial(F.d, m, F.b, F.BV(F.cur), DT::F64, F.ldq, W, DT::F64, F.ldq,
                           h->part.d(), chunks, gate, s));
  HIPCHK(launch_reduce_partials(chunks, m, F.b, h->part.d(), 1.0, beta, Hcol, F.ldh, -1.0,
                                h->hz.d(), F.b, gate, s));
  HIPCHK(launch_nn(F.d, m, F.b, F.V(F.cur), DT::F64, F.ldq, h->hz.d(), F.b, 1.0, W, DT::F64,
                   F.ldq, W, DT::F64, F.ldq, gate, s));
  if (U != nullptr)
    HIPCHK(launch_nn(F.d, m, F.b, F.BV(F.cur), DT::F64, F.ldq, h->hz.d(), F.b, 1.0, U, DT::F64,
                     F.ldq, U, DT::F64, F.ldq, gate, s));
  return EDA_OK;
}

// One Cholesky QR pass in <,>_W of the cols-column block W (U = exp(S_W) W,
// both ld ldq): G = W^T U = R^T R, Vo = W R^{-1}, Uo = U R^{-1} (in place
// allowed).  Rout (when given) receives R Rprev.
eda_status chol_pass(const AForm& F, int64_t cols, const double* W, const double* U, double* Vo,
                     double* Uo, const double* Rprev, double* Rout, int64_t ldro, int* flag,
                     const int* gate) {
  eda_handle h = F.h;
  hipStream_t s = h->stream;
  const int64_t chunks = tn_chunks(F.d, cols, cols);
  STCHK(ensure(h, h->part, (size_t)chunks * cols * cols * 8));
  const bool fused = cols <= 16;
  HIPCHK(launch_tn_partial(F.d, cols, cols, W, DT::F64, F.ldq, U, DT::F64, F.ldq, h->part.d(),
                           chunks, gate, s));
  if (!fused)
    HIPCHK(launch_reduce_partials(chunks, cols, cols, h->part.d(), 1.0, 0.0, h->Gs.d(), cols, 0.0,
                                  nullptr, 0, gate, s));
  HIPCHK(launch_chol(cols, h->Gs.d(), cols, h->Rinv.d(), cols, Rprev, cols, Rout, ldro, nullptr, 0,
                     0, 1e-4, flag, gate, s, fused ? h->part.d() : nullptr, chunks));
  HIPCHK(launch_nn(F.d, cols, cols, W, DT::F64, F.ldq, h->Rinv.d(), cols, 0.0, nullptr, DT::F64,
                   F.ldq, Vo, DT::F64, F.ldq, gate, s));
  HIPCHK(launch_nn(F.d, cols, cols, U, DT::F64, F.ldq, h->Rinv.d(), cols, 0.0, nullptr, DT::F64,
                   F.ldq, Uo, DT::F64, F.ldq, gate, s));
  return EDA_OK;
}

// Block step m: from V[:, 0:m+b] (current block V[:, m:m+b]) build
// V[:, m+b:m+2b] (and BV) and column block m of H.  Flag slots: 0 = this
// step's norm loss (bit 0) or deflation (bit 1) in the first factorisation,
// folded into slot 1 at the end of the step; 5 = a later factorisation that
// was not positive definite.
eda_status step(const AForm& F, int64_t m, bool repair) {
  eda_handle h = F.h;
  hipStream_t s = h->stream;
  const int64_t b = F.b, ldq = F.ldq, ldh = F.ldh, d = F.d;
  double* W = h->af[kW].d();
  double* Z = h->af[kZ].d();
  int* flags = h->flags.i();
  double* Hcol = F.H(F.cur) + m * ldh;
  STCHK(apply_a(F, b, F.V(F.cur) + (size_t)m * ldq, ldq, W, ldq));
  STCHK(project(F, m + b, W, nullptr, Hcol, 0.0, nullptr));
  STCHK(project(F, m + b, W, nullptr, Hcol, 1.0, nullptr));
  STCHK(apply_w(F, b, W, ldq, Z, ldq));
  double* Vn = F.V(F.cur) + (size_t)(m + b) * ldq;
  double* Bn = F.BV(F.cur) + (size_t)(m + b) * ldq;
  {
    // first factorisation rank revealing, with the norm-loss test against
    // the projection coefficients
    const int64_t chunks = tn_chunks(d, b, b);
    const bool fused = b <= 16;
    HIPCHK(launch_tn_partial(d, b, b, W, DT::F64, ldq, Z, DT::F64, ldq, h->part.d(), chunks,
                             nullptr, s));
    if (!fused)
      HIPCHK(launch_reduce_partials(chunks, b, b, h->part.d(), 1.0, 0.0, h->Gs.d(), b, 0.0,
                                    nullptr, 0, nullptr, s));
    HIPCHK(launch_pchol(b, h->Gs.d(), b, Hcol, m + b, ldh, 1e-13, 1e-4, false, h->Rinv.d(), b,
                        h->R1.d(), b, h->mask.i(), flags, s, fused ? h->part.d() : nullptr,
                        chunks));
    HIPCHK(launch_nn(d, b, b, W, DT::F64, ldq, h->Rinv.d(), b, 0.0, nullptr, DT::F64, ldq, Vn,
                     DT::F64, ldq, nullptr, s));
    HIPCHK(launch_nn(d, b, b, Z, DT::F64, ldq, h->Rinv.d(), b, 0.0, nullptr, DT::F64, ldq, Bn,
                     DT::F64, ldq, nullptr, s));
  }
  // R = R2 R1 -> H[m+b:m+2b, m:m+b]
  STCHK(chol_pass(F, b, Vn, Bn, Vn, Bn, h->R1.d(), Hcol + m + b, ldh, flags + 5, nullptr));
  if (repair) {
    // runs only when slot 0 was raised: project the new block again and
    // re-factor it (its coupling in H is left as it was)
    STCHK(project(F, m + b, Vn, Bn, nullptr, 0.0, flags));
    STCHK(project(F, m + b, Vn, Bn, nullptr, 0.0, flags));
    STCHK(chol_pass(F, b, Vn, Bn, Vn, Bn, nullptr, nullptr, 0, flags + 5, flags));
    STCHK(chol_pass(F, b, Vn, Bn, Vn, Bn, nullptr, nullptr, 0, flags + 5, flags));
  }
  HIPCHK(launch_flag_fold(flags, s));
  return EDA_OK;
}

// Rayleigh-Ritz on the leading m x m block of H (synchronous): top `cnt`
// Ritz values (descending) and residual estimates on the host, flags too.
// With cnt < kk (no restart follows) only cnt eigenvectors are formed, and
// those of eigenvalues closer than 1e-3 ||T|| are orthonormalised together
// only when closer than 1e-8 ||T|| (the final vectors are orthonormalised
// again).
eda_status ritz(const AForm& F, int64_t m, int64_t cnt, double* theta, double* est, int* fl) {
  eda_handle h = F.h;
  hipStream_t s = h->stream;
  const int64_t mm = F.mm;
  const bool keep = cnt >= F.kk;
  HIPCHK(launch_symmetrize(m, F.H(F.cur), F.ldh, h->T.d(), mm, s));
  HIPCHK(launch_syev(1, m, nullptr, h->T.d(), mm, 0, h->wT.d(), 0, h->S.d(), mm, 0,
                     std::min<int64_t>(m, keep ? F.kk : cnt), h->syev_work.d(), s,
                     keep ? 0.0 : 1e-8));
  const double* Bm = F.H(F.cur) + m + (m - F.b) * F.ldh;
  HIPCHK(launch_ritz_estimates(m, F.b, cnt, h->wT.d(), h->S.d(), mm, Bm, F.ldh, h->dtheta.d(),
                               h->dres.d(), s));
  HIPCHK(hipMemcpyAsync(theta, h->dtheta.d(), cnt * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(est, h->dres.d(), cnt * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(fl, h->flags.i(), 8 * sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return EDA_OK;
}

}  // namespace

namespace eda {

eda_status solve_aform(eda_handle h, int32_t t, double tol, const eda_solve_opts& o, double* ritz_out,
                       double* ritz_log, double* X, int64_t ldx, double* resid, eda_info* info) {
  if (o.krylov_dtype != EDA_F64)
    return fail(h, EDA_ERR_ARG, "the Arnoldi form runs in float64 (krylov_dtype EDA_F64)");
  if (h->normW > 12.0 * std::log(10.0))
    return fail(h, EDA_ERR_ARG,
                "||S_W|| = %.3g: exp(S_W) is too ill-conditioned for the Arnoldi form", h->normW);
  STCHK(ensure_arnoldi_core(h));
  AForm F;
  F.h = h;
  F.d = h->d;
  F.n = h->n;
  F.k = h->k;
  F.b = o.block > 0 ? o.block : 8;
  F.t = t;
  F.ldq = h->ldp;
  const int64_t b = F.b, d = F.d;
  if (b > 8) return fail(h, EDA_ERR_ARG, "block width must be in [1, 8]");
  // basis columns at most mmax + b, below the dimension n - 1 + b of the
  // invariant hull of the start block
  const int64_t cap = ((h->n - 1 - b) / b) * b;
  int64_t mmax = o.max_basis;
  if (mmax <= 0) {
    mmax = round_up(std::max<int64_t>(2 * t + 2 * b, t + 6 * b), b);
    mmax = std::min<int64_t>(mmax, std::min<int64_t>(cap, std::min<int64_t>(d, 2048 - b)));
  }
  if (mmax < t + 2 * b || mmax > d || mmax + b > 2048 || mmax > cap)
    return fail(h, EDA_ERR_ARG,
                "the Arnoldi form needs t + 2b <= max_basis <= %lld (n - 1 - b rounded down to "
                "a multiple of b); max_basis = %lld",
                (long long)cap, (long long)mmax);
  F.mmax = mmax;
  F.ldh = mmax + b;
  F.mm = mmax + b;
  F.kk = std::max<int64_t>(t, std::min<int64_t>(t + b, mmax - 2 * b));
  const int64_t ldq = F.ldq, ldh = F.ldh, mm = F.mm, kk = F.kk;
  const int64_t max_iter = o.max_iter > 0 ? o.max_iter : 4000;
  const int64_t check_every = o.check_every > 0 ? o.check_every : 2;
  if (o.start_block != nullptr && o.ld_start < d)
    return fail(h, EDA_ERR_ARG, "ld_start must be >= d");
  hipStream_t s = h->stream;

  for (int q = 0; q < 2; ++q) {
    STCHK(ensure(h, h->af[q ? kV1 : kV0], (size_t)ldq * mm * 8));
    STCHK(ensure(h, h->af[q ? kB1 : kB0], (size_t)ldq * mm * 8));
    STCHK(ensure(h, h->af[q ? kH1 : kH0], (size_t)ldh * ldh * 8));
  }
  const int64_t wcols = std::max<int64_t>(b, t);
  STCHK(ensure(h, h->af[kW], (size_t)ldq * wcols * 8));
  STCHK(ensure(h, h->af[kZ], (size_t)ldq * wcols * 8));
  STCHK(ensure(h, h->af[kG], (size_t)t * t * 8));
  STCHK(ensure(h, h->af[kGp], (size_t)h->n * h->n * 8));
  STCHK(ensure(h, h->T, (size_t)mm * mm * 8));
  STCHK(ensure(h, h->wT, (size_t)mm * 8));
  STCHK(ensure(h, h->S, (size_t)mm * mm * 8));
  STCHK(ensure(h, h->Sd, (size_t)mm * kk * 8));
  STCHK(ensure(h, h->dtheta, (size_t)(kk + 8) * 8));
  STCHK(ensure(h, h->dres, (size_t)(kk + 8) * 8));
  STCHK(ensure(h, h->syev_work, syev_work_bytes(mm)));
  STCHK(ensure(h, h->flags, 64));
  STCHK(ensure(h, h->mask, 128 * sizeof(int)));
  {
    const int64_t bt = std::max<int64_t>(b, t);
    const int64_t shapes[][2] = {{h->N, bt}, {mm, b}, {b, b}, {t, t}};
    size_t pmax = 0;
    for (const auto& sh : shapes)
      pmax = std::max(pmax, (size_t)tn_chunks(d, sh[0], sh[1]) * sh[0] * sh[1] * 8);
    STCHK(ensure(h, h->part, pmax));
    STCHK(ensure(h, h->Ysm, (size_t)h->N * bt * 8));
    STCHK(ensure(h, h->Zsm, (size_t)h->N * bt * 8));
    STCHK(ensure(h, h->hz, (size_t)mm * bt * 8));
    STCHK(ensure(h, h->Gs, (size_t)bt * bt * 8));
    STCHK(ensure(h, h->Rinv, (size_t)bt * bt * 8));
    STCHK(ensure(h, h->R1, (size_t)bt * bt * 8));
  }
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, s));
  STCHK(build_w_core(h, 1.0, h->af[kGp].d()));
  double* W = h->af[kW].d();
  double* Z = h->af[kZ].d();

  std::vector<double> theta(kk + 8), est(kk + 8);
  int fl[8];
  int64_t m = 0, iters = 0, restarts = 0, ops = 0;
  bool conv = false;
  const double u64 = 0x1.0p-53;
  auto converged = [&]() {
    const double th1 = theta[0];
    for (int64_t i = 0; i < t; ++i) {
      const double thi = theta[i];
      if (!(thi > 0.0) || !std::isfinite(est[i])) return false;
      const double tol_i = std::max(tol, 10.0 * u64 * th1 / thi);
      const double r = (o.resmode == EDA_RES_REL_THETA) ? est[i] / thi : est[i] / th1;
      if (!(r <= tol_i)) return false;
    }
    return true;
  };
  // The re-projection after a flagged block is left out away from the hull
  // dimension; a flag raised there anyway is seen at the next check and the
  // solve is started again with it in every step.
  const int64_t sat = h->n - 1 + b;
  bool safe = std::getenv("EDA_ALWAYS_REPAIR") != nullptr;
  bool checked_last = false;
  for (int attempt = 0;; ++attempt) {
    m = iters = restarts = 0;
    ops = b;
    F.cur = 0;
    checked_last = false;
    HIPCHK(launch_fill_i32(16, 0, h->flags.i(), s));
    for (int q = 0; q < 2; ++q) HIPCHK(launch_fill(ldh * ldh, 0.0, F.H(q), s));
    // start block: a Gaussian (or the given) block, Cholesky QR in <,>_W twice
    if (o.start_block != nullptr)
      HIPCHK(launch_copy2d(d, b, o.start_block, DT::F64, o.ld_start, W, DT::F64, ldq, s));
    else
      HIPCHK(launch_randn(d, b, o.seed, W, ldq, s));
    STCHK(apply_w(F, b, W, ldq, Z, ldq));
    STCHK(chol_pass(F, b, W, Z, F.V(0), F.BV(0), nullptr, nullptr, 0, h->flags.i() + 5, nullptr));
    STCHK(chol_pass(F, b, F.V(0), F.BV(0), F.V(0), F.BV(0), nullptr, nullptr, 0,
                    h->flags.i() + 5, nullptr));
    bool redo = false;
    while (true) {
      const bool repair = safe || (m + 3 * b >= sat);
      STCHK(step(F, m, repair));
      m += b;
      ++iters;
      ops += b;
      checked_last = false;
      const bool need_restart = (m + b > mmax);
      const bool can_check = (m >= t + b) || need_restart;
      if (!(can_check && (iters % check_every == 0 || need_restart || iters >= max_iter)))
        continue;
      const int64_t cnt = need_restart ? kk : t;
      STCHK(ritz(F, m, cnt, theta.data(), est.data(), fl));
      checked_last = true;
      if ((fl[1] & 2) || fl[5]) {
        if (std::getenv("EDA_LOG") != nullptr)
          std::fprintf(stderr, "[eda] aform m=%lld flags %d %d\n", (long long)m, fl[1], fl[5]);
        return fail(h, EDA_ERR_NOCONV,
                    "a block lost rank in the exp(S_W) inner product before convergence");
      }
      if (fl[1] != 0 && !safe) {
        redo = true;
        break;
      }
      for (int64_t i = 0; i < cnt; ++i)
        if (!std::isfinite(theta[i]) || !std::isfinite(est[i]))
          return fail(h, EDA_ERR_NONFINITE, "non-finite Ritz pair");
      if (converged()) {
        conv = true;
        break;
      }
      if (iters >= max_iter) break;
      if (need_restart) {
        // thick restart: V S_kk, BV S_kk and the next block
        HIPCHK(launch_gather_desc(m, kk, h->S.d(), mm, h->Sd.d(), kk, s));
        const int nxt = 1 - F.cur;
        HIPCHK(launch_nn(d, m, kk, F.V(F.cur), DT::F64, ldq, h->Sd.d(), kk, 0.0, nullptr, DT::F64,
                         ldq, F.V(nxt), DT::F64, ldq, nullptr, s));
        HIPCHK(launch_nn(d, m, kk, F.BV(F.cur), DT::F64, ldq, h->Sd.d(), kk, 0.0, nullptr,
                         DT::F64, ldq, F.BV(nxt), DT::F64, ldq, nullptr, s));
        HIPCHK(launch_copy2d(d, b, F.V(F.cur) + (size_t)m * ldq, DT::F64, ldq,
                             F.V(nxt) + (size_t)kk * ldq, DT::F64, ldq, s));
        HIPCHK(launch_copy2d(d, b, F.BV(F.cur) + (size_t)m * ldq, DT::F64, ldq,
                             F.BV(nxt) + (size_t)kk * ldq, DT::F64, ldq, s));
        double* Hn = F.H(nxt);
        HIPCHK(launch_fill(ldh * ldh, 0.0, Hn, s));
        HIPCHK(launch_set_diag(kk, h->dtheta.d(), Hn, ldh, s));
        HIPCHK(launch_restart_coupling(m, b, kk, F.H(F.cur) + m + (m - b) * ldh, ldh, h->Sd.d(),
                                       kk, Hn, ldh, s));
        F.cur = nxt;
        m = kk;
        ++restarts;
        checked_last = false;
      }
    }
    if (!redo) break;
    safe = true;
  }
  if (m < t) return fail(h, EDA_ERR_NOCONV, "basis smaller than t at the iteration limit");
  if (!checked_last) STCHK(ritz(F, m, t, theta.data(), est.data(), fl));

  // x = V s (descending); D = e^{-s} A x - theta x; ||r||^2 = D^T exp(S_W) D
  HIPCHK(launch_gather_desc(m, t, h->S.d(), mm, h->Sd.d(), t, s));
  HIPCHK(launch_nn(d, m, t, F.V(F.cur), DT::F64, ldq, h->Sd.d(), t, 0.0, nullptr, DT::F64, ldq, X,
                   DT::F64, ldx, nullptr, s));
  STCHK(apply_a(F, t, X, ldx, W, ldq));
  HIPCHK(launch_ritz_residual(d, t, W, ldq, X, ldx, h->dtheta.d(), W, ldq, h->dres.d(), s));
  STCHK(apply_w(F, t, W, ldq, Z, ldq));
  ops += 2 * t;
  {
    const int64_t chunks = tn_chunks(d, t, t);
    STCHK(ensure(h, h->part, (size_t)chunks * t * t * 8));
    HIPCHK(launch_tn_partial(d, t, t, W, DT::F64, ldq, Z, DT::F64, ldq, h->part.d(), chunks,
                             nullptr, s));
    HIPCHK(launch_reduce_partials(chunks, t, t, h->part.d(), 1.0, 0.0, h->af[kG].d(), t, 0.0,
                                  nullptr, 0, nullptr, s));
  }
  std::vector<double> G((size_t)t * t);
  HIPCHK(hipMemcpyAsync(theta.data(), h->dtheta.d(), t * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(G.data(), h->af[kG].d(), (size_t)t * t * 8, hipMemcpyDeviceToHost, s));
  // orthonormalise in decreasing-lambda order (Cholesky QR twice), fix signs
  STCHK(orthonormalise(h, t, X, ldx, ldq));
  HIPCHK(hipEventRecord(e1, s));
  HIPCHK(hipStreamSynchronize(s));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);

  bool range_err = false, ok = true;
  for (int64_t i = 0; i < t; ++i) {
    const double th = theta[i];
    const double rn = std::sqrt(std::max(0.0, G[i + i * t]));
    if (!(th > 0.0)) {
      range_err = true;
      ritz_log[i] = -INFINITY;
      ritz_out[i] = 0.0;
      resid[i] = INFINITY;
      continue;
    }
    ritz_log[i] = h->shiftB + std::log(th);
    ritz_out[i] = std::exp(ritz_log[i]);
    resid[i] = (o.resmode == EDA_RES_REL_THETA) ? rn / th : rn / theta[0];
    if (!(resid[i] <= std::max(tol, 10.0 * u64 * theta[0] / th))) ok = false;
  }
  if (info != nullptr) {
    std::memset(info, 0, sizeof(*info));
    info->iters = (int32_t)iters;
    info->restarts = (int32_t)restarts;
    info->flags = (t > h->k - 1 ? EDA_WARN_DEGENERATE : 0) | (safe ? EDA_WARN_REPAIRED : 0);
    info->ops = ops;
    // per block step: P^T V and P Y over the n + k columns of P for the
    // product with A, and again over the n columns of H_W for exp(S_W)
    info->bytes_moved = (double)iters * 2.0 * d * (h->N + h->n) * 8.0;
    info->t_prepare_ms = prepare_time_ms(h);
    info->t_krylov_ms = ms;
    info->shift_s = h->shiftB;
  }
  if (range_err) return fail(h, EDA_ERR_RANGE, "a Ritz value underflowed after the shift");
  if (!conv) return fail(h, EDA_ERR_NOCONV, "max_iter reached before convergence");
  if (!ok)
    return fail(h, EDA_ERR_NOCONV, "the explicit residual of the Ritz pairs exceeds the tolerance");
  return EDA_OK;
}

}  // namespace eda
