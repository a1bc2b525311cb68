// libeda host library, part 2: eda_solve.
//
// Block Lanczos with thick restart on the shifted symmetric operator
// e^{-s} M, M = exp(-S_W/2) exp(S_B) exp(-S_W/2) (eqs. (3.13)-(3.16)), which
// is step 5 of Algorithm 3 in its Lanczos form, followed by
//   * an explicit float64 check, and if needed float64 refinement passes
//     (Rayleigh-Ritz on span[Y, R] with the float64 operator), and
//   * the back-transform x = exp(-S_W/2) y of eq. (3.14) with
//     orthonormalisation in decreasing-lambda order (Algorithm 3, step 6).
// The Krylov phase may run on narrower operands: the operator P = [H_W H_B]
// in the storage type chosen at eda_prepare (float64, float32, bfloat16) and
// the basis in float64 or float32.  It then stops at the accuracy those
// types can reach, and the float64 stage takes the pairs to the tolerance.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "host_internal.h"

using namespace eda;

namespace {

double unit_roundoff(DT t) {
  switch (t) {
    case DT::F64: return 0x1.0p-53;
    case DT::F32: return 0x1.0p-24;
    case DT::BF16: return 0x1.0p-8;
    default: return 0x1.0p-4;  // FP8 E4M3
  }
}

struct Solver {
  eda_handle h;
  int64_t d, ldq, b, mmax, ldh, t, kk;
  DT qdt;       // basis type of the Krylov phase
  int cur = 0;  // which of the two basis/H buffers is live
  // float64 P: the products keep P^T Q (h->PQ[cur], row-major, ld ldpq)
  bool track = false;
  int64_t ldpq = 0;
  char* Q() const { return h->Q[cur].c(); }
  char* Qc(int64_t j) const { return Q() + (size_t)j * ldq * dt_size(qdt); }
  double* H() const { return h->H[cur].d(); }
};

}  // namespace

namespace eda {

eda_status cholqr_pass(eda_handle h, int64_t d, int64_t cols, const void* X, DT xdt, int64_t ldx,
                       void* Xout, int64_t ldxo, const double* Rprev, double* Rout, int64_t ldro,
                       const double* hcol, int64_t mrows, int64_t ldhc, const int* gate,
                       int* flag) {
  int64_t chunks = tn_chunks(d, cols, cols);
  STCHK(ensure(h, h->Gs, (size_t)cols * cols * 8));
  STCHK(ensure(h, h->Rinv, (size_t)cols * cols * 8));
  // for a narrow block the Cholesky kernel sums the chunk partials of
  // X^T X itself; wide float64 blocks (Ritz blocks) take the matrix-core
  // Gram, others the tn partials and the parallel reduction
  const bool fused = cols <= 16;
  const bool gram = !fused && cols >= 48 && gate == nullptr && xdt == DT::F64 && ldx % 2 == 0 &&
                    ((uintptr_t)X % 16) == 0;
  if (gram) {
    chunks = gram_block_chunks(d, cols);
    STCHK(ensure(h, h->part, (size_t)chunks * cols * cols * 8));
    HIPCHK(launch_gram_block(d, cols, (const double*)X, ldx, h->part.d(), chunks, h->Gs.d(), cols,
                             h->stream));
  } else {
    STCHK(ensure(h, h->part, (size_t)chunks * cols * cols * 8));
    HIPCHK(launch_tn_partial(d, cols, cols, X, xdt, ldx, X, xdt, ldx, h->part.d(), chunks, gate,
                             h->stream));
    if (!fused)
      HIPCHK(launch_reduce_partials(chunks, cols, cols, h->part.d(), 1.0, 0.0, h->Gs.d(), cols,
                                    0.0, nullptr, 0, gate, h->stream));
  }
  HIPCHK(launch_chol(cols, h->Gs.d(), cols, h->Rinv.d(), cols, Rprev, cols, Rout, ldro, hcol,
                     mrows, ldhc, 1e-4, flag, gate, h->stream, fused ? h->part.d() : nullptr,
                     chunks));
  HIPCHK(launch_nn(d, cols, cols, X, xdt, ldx, h->Rinv.d(), cols, 0.0, nullptr, xdt, ldx, Xout,
                   xdt, ldxo, gate, h->stream));
  return EDA_OK;
}

eda_status cgs_pass(eda_handle h, int64_t d, int64_t m, const void* Q, DT qdt, int64_t ldq,
                    void* W, int64_t ldw, int64_t b, double* Hcol, int64_t ldh, double beta,
                    const int* gate) {
  const int64_t chunks = tn_chunks(d, m, b);
  STCHK(ensure(h, h->part, (size_t)chunks * m * b * 8));
  STCHK(ensure(h, h->hz, (size_t)m * b * 8));
  HIPCHK(launch_tn_partial(d, m, b, Q, qdt, ldq, W, qdt, ldw, h->part.d(), chunks, gate,
                           h->stream));
  HIPCHK(launch_reduce_partials(chunks, m, b, h->part.d(), 1.0, beta, Hcol, ldh, -1.0, h->hz.d(),
                                b, gate, h->stream));
  HIPCHK(launch_nn(d, m, b, Q, qdt, ldq, h->hz.d(), b, 1.0, W, qdt, ldw, W, qdt, ldw, gate,
                   h->stream));
  return EDA_OK;
}

}  // namespace eda

namespace {

// Block step: from the basis Q[:, 0:m+b] (current block Q[:, m:m+b]) build
// Q[:, m+b:m+2b] and column block m of H.
// W = e^{-s} M V_j in the Krylov-phase types.
eda_status lanczos_op(Solver& S, int64_t m) {
  eda_handle h = S.h;
  // e^{-s} is read from the device, so a captured step stays valid when a
  // later preparation changes the shift
  // W goes straight into the slot of the next block, Q[:, m+b:m+2b]
  void* W = S.Qc(m + S.b);
  if (!S.track)
    return expop(h, false, 0, h->N, h->CM.d(), h->N, h->alphaB, S.b, S.Qc(m), S.qdt, S.ldq, W,
                 S.qdt, S.ldq, h->alphaB_dev.d());
  // P^T V_m goes to columns m .. m+b of P^T Q
  double* pq = h->PQ[S.cur].d() + m;
  STCHK(expop_first(h, false, 0, h->N, S.b, S.Qc(m), S.qdt, S.ldq, pq, S.ldpq));
  return expop_second(h, false, 0, h->N, h->CM.d(), h->N, h->alphaB, S.b, S.Qc(m), S.qdt,
                      S.ldq, W, S.qdt, S.ldq, h->alphaB_dev.d(), pq, S.ldpq);
}

// The rest of the block step: orthonormalise W into the next block and
// record its coefficients in H.
eda_status lanczos_orth(Solver& S, int64_t m, bool repair) {
  eda_handle h = S.h;
  const int64_t d = S.d, b = S.b, ldq = S.ldq, ldh = S.ldh;
  const DT qdt = S.qdt;
  double* H = S.H();
  // W (the product) already sits in the slot of the next block
  char* Qn = S.Qc(m + b);
  void* W = Qn;
  // without the repair pass, a raised flag goes to the sticky slot 2 that
  // the host reads at every check
  int* flags = repair ? h->flags.i() : h->flags.i() + 2;
  // CGS2 against Q[:, 0:m+b], first pass
  double* Hcol = H + m * ldh;
  STCHK(cgs_pass(h, d, m + b, S.Q(), qdt, ldq, W, ldq, b, Hcol, ldh, 0.0, nullptr));
  // Second pass and the Gram matrix of its result from one product:
  // [Q W]^T W = [h2; W^T W] (W adjacent to Q), h2 added to H, and
  // (W - Q h2)^T (W - Q h2) = W^T W - h2^T h2 for orthonormal Q, formed by
  // the Cholesky kernel (h2 is of the order of the rounding of the first
  // pass, so the difference loses nothing).
  {
    const int64_t chunks = tn_chunks(d, m + 2 * b, b);
    HIPCHK(launch_tn_partial(d, m + 2 * b, b, S.Q(), qdt, ldq, W, qdt, ldq, h->part.d(), chunks,
                             nullptr, h->stream));
    HIPCHK(launch_reduce_partials(chunks, m + 2 * b, b, h->part.d(), 1.0, 1.0, Hcol, ldh, -1.0,
                                  h->hz.d(), b, nullptr, h->stream, m + b, h->Gs.d(), b));
    HIPCHK(launch_nn(d, m + b, b, S.Q(), qdt, ldq, h->hz.d(), b, 1.0, W, qdt, ldq, W, qdt, ldq,
                     nullptr, h->stream));
  }
  // Block orthonormalisation, R = R2 R1 going to H[m+b:m+2b, m:m+b].
  // Pass 1 is rank revealing: directions along which the Krylov space has
  // become invariant are deflated and replaced by fresh random directions
  // with zero coupling (their rows of R1 are zero).
  HIPCHK(launch_pchol(b, h->Gs.d(), b, Hcol, m + b, ldh, 1e-13, 1e-4, false, h->Rinv.d(), b,
                      h->R1.d(), b, h->mask.i(), flags, h->stream, nullptr, 0, h->hz.d(),
                      m + b));
  // Q_n = W R1^{-1} in place (b <= 16 columns: one workgroup column reads
  // all of a row before writing it); the product writes the random
  // replacement columns
  HIPCHK(launch_nn(d, b, b, W, qdt, ldq, h->Rinv.d(), b, 0.0, nullptr, qdt, ldq, Qn, qdt, ldq,
                   nullptr, h->stream, false, nullptr, nullptr, h->mask.i(),
                   0x5eed0000ull + (uint64_t)m));
  STCHK(cholqr_pass(h, d, b, Qn, qdt, ldq, Qn, ldq, h->R1.d(), H + (m + b) + m * ldh, ldh,
                    nullptr, 0, 0, nullptr, flags));
  if (!repair) return EDA_OK;
  // repair (only runs when the flag was raised): re-orthogonalise the new block
  STCHK(cgs_pass(h, d, m + b, S.Q(), qdt, ldq, Qn, ldq, b, nullptr, 0, 0.0, flags));
  STCHK(cgs_pass(h, d, m + b, S.Q(), qdt, ldq, Qn, ldq, b, nullptr, 0, 0.0, flags));
  STCHK(cholqr_pass(h, d, b, Qn, qdt, ldq, Qn, ldq, nullptr, nullptr, 0, nullptr, 0, 0, flags,
                    nullptr));
  STCHK(cholqr_pass(h, d, b, Qn, qdt, ldq, Qn, ldq, nullptr, nullptr, 0, nullptr, 0, 0, flags,
                    nullptr));
  HIPCHK(launch_flag_fold(flags, h->stream));
  return EDA_OK;
}

// Captures one call of f (launches on h->stream) into an executable graph,
// recorded on the handle's capture stream.
template <class F>
eda_status capture(eda_handle h, F f, hipGraphExec_t* exec) {
  if (h->cap == nullptr) HIPCHK(hipStreamCreateWithFlags(&h->cap, hipStreamNonBlocking));
  hipStream_t keep = h->stream;
  h->stream = h->cap;
  hipError_t e = hipStreamBeginCapture(h->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) {
    h->stream = keep;
    return fail(h, EDA_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
  }
  const eda_status st = f();
  hipGraph_t g = nullptr;
  e = hipStreamEndCapture(h->cap, &g);
  h->stream = keep;
  if (st != EDA_OK) {
    if (g != nullptr) (void)hipGraphDestroy(g);
    return st;
  }
  if (e != hipSuccess) return fail(h, EDA_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(h, EDA_ERR_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
  return EDA_OK;
}

// Block step m.  With graphs, the product and the orthonormalisation of a
// given (m, basis buffer) are captured once per solver configuration and
// replayed; the product stays bracketed by the timing events.
eda_status lanczos_step(Solver& S, int64_t m, bool graphs, bool repair) {
  eda_handle h = S.h;
  if (h->op_used + 2 > h->op_ev.size()) {
    for (int q = 0; q < 64; ++q) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      h->op_ev.push_back(e);
    }
  }
  hipGraphExec_t gop = nullptr, grest = nullptr;
  if (graphs) {
    for (const auto& g : h->graphs)
      if (g.m == m && g.cur == S.cur && g.repair == repair) {
        gop = g.op;
        grest = g.rest;
      }
    if (gop == nullptr) {
      STCHK(capture(h, [&]() { return lanczos_op(S, m); }, &gop));
      STCHK(capture(h, [&]() { return lanczos_orth(S, m, repair); }, &grest));
      h->graphs.push_back(StepGraph{m, S.cur, repair, gop, grest});
    }
  }
  HIPCHK(hipEventRecord(h->op_ev[h->op_used], h->stream));
  if (graphs)
    HIPCHK(hipGraphLaunch(gop, h->stream));
  else
    STCHK(lanczos_op(S, m));
  HIPCHK(hipEventRecord(h->op_ev[h->op_used + 1], h->stream));
  h->op_used += 2;
  if (graphs)
    HIPCHK(hipGraphLaunch(grest, h->stream));
  else
    STCHK(lanczos_orth(S, m, repair));
  return EDA_OK;
}

void log_pairs(const char* tag, int64_t m, int64_t cnt, const double* theta, const double* est) {
  std::fprintf(stderr, "[eda] %s m=%lld theta:", tag, (long long)m);
  for (int64_t i = 0; i < cnt; ++i) std::fprintf(stderr, " %.6e", theta[i]);
  std::fprintf(stderr, "\n[eda]   res:");
  for (int64_t i = 0; i < cnt; ++i) std::fprintf(stderr, " %.2e", est[i]);
  std::fprintf(stderr, "\n");
}

// Cluster tolerance of the eigensolver for checks whose Ritz vectors are
// not kept in a restarted basis: their vectors only give residual estimates
// (or are orthonormalised again at the end), so eigenvectors of eigenvalues
// closer than 1e-3 ||T|| need not be orthonormalised together, only those
// closer than 1e-8 ||T|| (orthogonal to about u / 1e-8 otherwise).
constexpr double kCheckCtol = 1e-8;

// Rayleigh-Ritz on Q[:, 0:m]: eigenpairs of sym(H[0:m,0:m]); returns the top
// `cnt` Ritz values (descending) and residual estimates on the host.
eda_status rayleigh_ritz(Solver& S, int64_t m, int64_t nvec, int64_t cnt, double* theta,
                         double* est, int* flag0 = nullptr, double ctol = 0.0) {
  eda_handle h = S.h;
  const int64_t ldh = S.ldh, mm = S.mmax;
  HIPCHK(launch_symmetrize(m, S.H(), ldh, h->T.d(), mm, h->stream));
  HIPCHK(launch_syev(1, m, nullptr, h->T.d(), mm, 0, h->wT.d(), 0, h->S.d(), mm, 0, nvec,
                     h->syev_work.d(), h->stream, ctol));
  const double* Bm = S.H() + m + (m - S.b) * ldh;
  HIPCHK(launch_ritz_estimates(m, S.b, cnt, h->wT.d(), h->S.d(), mm, Bm, ldh, h->dtheta.d(),
                               h->dres.d(), h->stream));
  HIPCHK(hipMemcpyAsync(theta, h->dtheta.d(), cnt * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(est, h->dres.d(), cnt * 8, hipMemcpyDeviceToHost, h->stream));
  int f0 = 0;
  HIPCHK(hipMemcpyAsync(&f0, h->flags.i() + 2, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (flag0 != nullptr) *flag0 = f0;
  if (std::getenv("EDA_LOG") != nullptr) log_pairs("rr", m, cnt, theta, est);
  return EDA_OK;
}

// The same Rayleigh-Ritz, launched on the second stream after the work
// enqueued so far on the main stream; its Ritz values and estimates land in
// pinned memory and are read by rr_collect.  The block steps enqueued
// meanwhile on the main stream write only columns >= m of H and of the
// basis, which this reads nowhere.
eda_status rr_launch_async(Solver& S, int64_t m, int64_t nvec, int64_t cnt) {
  eda_handle h = S.h;
  const int64_t ldh = S.ldh, mm = S.mmax;
  hipStream_t a = h->aux;
  HIPCHK(hipEventRecord(h->ev_main, h->stream));
  HIPCHK(hipStreamWaitEvent(a, h->ev_main, 0));
  HIPCHK(launch_symmetrize(m, S.H(), ldh, h->T.d(), mm, a));
  HIPCHK(launch_syev(1, m, nullptr, h->T.d(), mm, 0, h->wT.d(), 0, h->S.d(), mm, 0, nvec,
                     h->syev_work.d(), a, kCheckCtol));
  const double* Bm = S.H() + m + (m - S.b) * ldh;
  HIPCHK(launch_ritz_estimates(m, S.b, cnt, h->wT.d(), h->S.d(), mm, Bm, ldh, h->dtheta.d(),
                               h->dres.d(), a));
  HIPCHK(hipMemcpyAsync(h->rr_pin, h->dtheta.d(), cnt * 8, hipMemcpyDeviceToHost, a));
  HIPCHK(hipMemcpyAsync(h->rr_pin + cnt, h->dres.d(), cnt * 8, hipMemcpyDeviceToHost, a));
  HIPCHK(hipMemcpyAsync(h->rr_pin + 2 * cnt, h->flags.i() + 2, sizeof(int), hipMemcpyDeviceToHost, a));
  HIPCHK(hipEventRecord(h->ev_rr, a));
  return EDA_OK;
}

eda_status rr_collect(Solver& S, int64_t m, int64_t cnt, double* theta, double* est, int* flag0) {
  eda_handle h = S.h;
  HIPCHK(hipEventSynchronize(h->ev_rr));
  std::memcpy(theta, h->rr_pin, cnt * 8);
  std::memcpy(est, h->rr_pin + cnt, cnt * 8);
  std::memcpy(flag0, h->rr_pin + 2 * cnt, sizeof(int));
  if (std::getenv("EDA_LOG") != nullptr) log_pairs("rr-async", m, cnt, theta, est);
  return EDA_OK;
}

}  // namespace

namespace eda {

eda_status rr_block(eda_handle h, int64_t d, int64_t ld, int64_t w, int64_t t, int64_t mm,
                    const double* B, const double* MB, double* Y, double* MY) {
  hipStream_t s = h->stream;
  const int64_t chunks = tn_chunks(d, w, w);
  HIPCHK(launch_tn_partial(d, w, w, B, DT::F64, ld, MB, DT::F64, ld, h->part.d(), chunks, nullptr,
                           s));
  HIPCHK(launch_reduce_partials(chunks, w, w, h->part.d(), 1.0, 0.0, h->S.d(), mm, 0.0, nullptr, 0,
                                nullptr, s));
  HIPCHK(launch_symmetrize(w, h->S.d(), mm, h->T.d(), mm, s));
  HIPCHK(launch_syev(1, w, nullptr, h->T.d(), mm, 0, h->wT.d(), 0, h->S.d(), mm, 0, t,
                     h->syev_work.d(), s));
  HIPCHK(launch_gather_desc(w, t, h->S.d(), mm, h->Sd.d(), t, s));
  HIPCHK(launch_desc_values(t, h->wT.d(), w, h->dtheta.d(), s));
  HIPCHK(launch_nn(d, w, t, B, DT::F64, ld, h->Sd.d(), t, 0.0, nullptr, DT::F64, ld, Y, DT::F64,
                   ld, nullptr, s));
  HIPCHK(launch_nn(d, w, t, MB, DT::F64, ld, h->Sd.d(), t, 0.0, nullptr, DT::F64, ld, MY, DT::F64,
                   ld, nullptr, s));
  return EDA_OK;
}

}  // namespace eda

namespace eda {

// x = exp(-S_W/2) y for the t Ritz vectors Y (float64, ld ldy), then
// orthonormalised in column order by Cholesky QR run twice (scratch with
// leading dimension ldw in h->Yb) and sign-fixed (eq. 3.14; Algorithm 3).
eda_status back_transform(eda_handle h, int64_t t, const double* Y, int64_t ldy, double* X,
                          int64_t ldx, int64_t ldw, bool ysm_ready) {
  // H_W is the leading n columns of P, so H_W^T Y is the leading n rows of P^T Y
  if (!ysm_ready) STCHK(expop_first(h, true, 0, h->n, t, Y, DT::F64, ldy));
  STCHK(expop_second(h, true, 0, h->n, h->Gh.d(), h->n, 1.0, t, Y, DT::F64, ldy, X, DT::F64,
                     ldx));
  return orthonormalise(h, t, X, ldx, ldw);
}

eda_status orthonormalise(eda_handle h, int64_t t, double* X, int64_t ldx, int64_t ldw) {
  const int64_t d = h->d;
  STCHK(ensure(h, h->Yb, (size_t)ldw * t * 8));
  STCHK(cholqr_pass(h, d, t, X, DT::F64, ldx, h->Yb.d(), ldw, nullptr, nullptr, 0, nullptr, 0, 0,
                    nullptr, nullptr));
  STCHK(cholqr_pass(h, d, t, h->Yb.d(), DT::F64, ldw, X, ldx, nullptr, nullptr, 0, nullptr, 0, 0,
                    nullptr, nullptr));
  HIPCHK(launch_sign_fix(d, t, X, ldx, h->stream));
  return EDA_OK;
}

}  // namespace eda

extern "C" eda_status eda_solve(eda_handle h, int32_t t, double tol, const eda_solve_opts* opt,
                                double* ritz, double* ritz_log, double* X, int64_t ldx,
                                double* resid, eda_info* info) {
  if (h == nullptr) return EDA_ERR_ARG;
  eda_solve_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opt != nullptr) o = *opt;
  if (!h->prepared) return fail(h, EDA_ERR_STATE, "eda_prepare has not succeeded");
  const int64_t d = h->d;
  if (t < 1 || t >= d) return fail(h, EDA_ERR_ARG, "need 1 <= t < d");
  if (t > 128) return fail(h, EDA_ERR_ARG, "t > 128 is not supported");
  if (!(tol > 0.0) || !std::isfinite(tol)) return fail(h, EDA_ERR_ARG, "tol must be positive");
  if (ritz == nullptr || ritz_log == nullptr || X == nullptr || resid == nullptr)
    return fail(h, EDA_ERR_ARG, "null output pointer");
  if (ldx < d) return fail(h, EDA_ERR_ARG, "ldx must be >= d");
  if (o.form != EDA_FORM_LANCZOS_M && o.form != EDA_FORM_ARNOLDI_A && o.form != EDA_FORM_JD_M)
    return fail(h, EDA_ERR_ARG, "unknown form");
  if (o.krylov_dtype != EDA_F64 && o.krylov_dtype != EDA_F32)
    return fail(h, EDA_ERR_ARG, "krylov_dtype (basis type) must be EDA_F64 or EDA_F32");
  if (o.refine_dtype != EDA_F64) return fail(h, EDA_ERR_ARG, "refine_dtype must be EDA_F64");
  if (o.resmode != EDA_RES_REL_THETA && o.resmode != EDA_RES_NORMWISE)
    return fail(h, EDA_ERR_ARG, "unknown residual mode");
  const int64_t b = o.block > 0 ? o.block : 8;
  if (b > 16) return fail(h, EDA_ERR_ARG, "block width must be in [1, 16]");
  int64_t mmax = o.max_basis;
  if (mmax <= 0) {
    mmax = std::max<int64_t>(2 * t + 2 * b, t + 6 * b);
    mmax = round_up(mmax, b);
    mmax = std::min<int64_t>(mmax, std::min<int64_t>(d, 2048 - b));
  }
  if (mmax < t + 2 * b || mmax > d || mmax + b > 2048)
    return fail(h, EDA_ERR_ARG, "max_basis=%lld must satisfy t+2b <= max_basis <= min(d, 2048-b)",
                (long long)mmax);
  const int64_t max_iter = o.max_iter > 0 ? o.max_iter : 4000;
  // check_every > 0: a Rayleigh-Ritz check every that many block steps;
  // 0: checks scheduled from the observed convergence rate (below)
  const int64_t check_every = o.check_every > 0 ? o.check_every : 0;
  if (o.start_block != nullptr && o.ld_start < d)
    return fail(h, EDA_ERR_ARG, "ld_start must be >= d");
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, X, "X"));
  if (o.start_block != nullptr) STCHK(check_dev_ptr(h, o.start_block, "start_block"));
  if (o.form == EDA_FORM_ARNOLDI_A) return solve_aform(h, t, tol, o, ritz, ritz_log, X, ldx, resid, info);
  if (o.form == EDA_FORM_JD_M) return solve_jd(h, t, tol, o, ritz, ritz_log, X, ldx, resid, info);

  const DT qdt = o.krylov_dtype == EDA_F32 ? DT::F32 : DT::F64;
  const bool mixed = (h->storage != EDA_F64) || (qdt != DT::F64);
  // Float64 passes after the Krylov phase (defaults: 16 after a narrow
  // phase, 2 as a safety net after a float64 one); negative: none, and no
  // float64 Rayleigh-Ritz either (the pairs of the Krylov phase are returned
  // with float64 residuals).
  const int64_t max_refine = o.max_refine > 0 ? o.max_refine : (o.max_refine < 0 ? -1 : (mixed ? 16 : 2));
  const double u_lo = std::max(unit_roundoff(dt_of(h->storage)), unit_roundoff(qdt));

  Solver S;
  S.h = h;
  S.d = d;
  S.ldq = h->ldp;
  S.b = b;
  S.mmax = mmax;
  S.ldh = mmax + b;
  S.t = t;
  S.qdt = qdt;
  S.kk = std::min<int64_t>(t + b, mmax - 2 * b);
  if (S.kk < t) S.kk = t;
  const int64_t ldq = S.ldq, ldh = S.ldh;
  const size_t qs = dt_size(qdt);
  const int64_t wz = std::min<int64_t>(t, d - t);          // refinement expansion width
  const int64_t mm = std::max<int64_t>(mmax, t + wz);      // leading dimension of T, S

  for (int q = 0; q < 2; ++q) {
    STCHK(ensure(h, h->Q[q], (size_t)ldq * (mmax + b) * qs));
    STCHK(ensure(h, h->H[q], (size_t)ldh * ldh * 8));
  }
  // With float64 P, P^T y of the final Ritz block follows from P^T Q by a
  // small product instead of a pass over P
  S.track = (h->storage == EDA_F64);
  S.ldpq = mmax + b;
  if (S.track)
    for (int q = 0; q < 2; ++q) STCHK(ensure(h, h->PQ[q], (size_t)h->N * S.ldpq * 8));
  STCHK(ensure(h, h->Wb, (size_t)ldq * b * qs));
  STCHK(ensure(h, h->T, (size_t)mm * mm * 8));
  STCHK(ensure(h, h->wT, (size_t)mm * 8));
  STCHK(ensure(h, h->S, (size_t)mm * mm * 8));
  STCHK(ensure(h, h->Sd, (size_t)std::max(mmax * S.kk, (t + wz) * t) * 8));
  STCHK(ensure(h, h->Yb, (size_t)ldq * std::max<int64_t>(t, b) * 8));
  // refinement blocks [Y | R] and [MY | MR], two of each, 2t columns apiece
  STCHK(ensure(h, h->refine, (size_t)8 * ldq * t * 8));
  STCHK(ensure(h, h->dtheta, (size_t)(S.kk + 8) * 8));
  STCHK(ensure(h, h->dres, (size_t)(S.kk + 8) * 8));
  STCHK(ensure(h, h->syev_work, syev_work_bytes(mm)));
  STCHK(ensure(h, h->flags, 64));
  STCHK(ensure(h, h->mask, 128 * sizeof(int)));
  {
    // size the shared workspaces once for every shape used below
    const int64_t bt = std::max<int64_t>(b, t);
    const int64_t shapes[][2] = {{h->N, b},  {mmax + b, b}, {b, b},   {h->N, t},
                                 {h->n, t},  {t, t},        {t, wz},  {wz, wz},
                                 {t + wz, t + wz}};
    size_t pmax = 0;
    for (const auto& sh : shapes)
      pmax = std::max(pmax, (size_t)tn_chunks(d, sh[0], sh[1]) * sh[0] * sh[1] * 8);
    STCHK(ensure(h, h->part, pmax));
    STCHK(ensure(h, h->Ysm, (size_t)h->N * bt * 8));
    STCHK(ensure(h, h->Zsm, (size_t)h->N * bt * 8));
    STCHK(ensure(h, h->hz, (size_t)std::max<int64_t>((mmax + b) * b, (int64_t)t * t) * 8));
    STCHK(ensure(h, h->Gs, (size_t)bt * bt * 8));
    STCHK(ensure(h, h->Rinv, (size_t)bt * bt * 8));
    const int64_t rb = std::max<int64_t>(b, std::min<int64_t>(wz, 64));  // pchol's R
    STCHK(ensure(h, h->R1, (size_t)rb * rb * 8));
  }

  // EDA_GRAPHS=1 replays the block steps from captured graphs (valid while
  // every buffer and size they bake in is unchanged).
  const char* genv = std::getenv("EDA_GRAPHS");
  const bool use_graphs = genv != nullptr && std::strcmp(genv, "1") == 0;
  {
    const uint64_t parts[] = {
        (uint64_t)(uintptr_t)h->alphaB_dev.p, (uint64_t)d, (uint64_t)h->N, (uint64_t)b, (uint64_t)qdt, (uint64_t)ldq,
        (uint64_t)ldh, (uint64_t)mmax, (uint64_t)h->storage, (uint64_t)(uintptr_t)h->Q[0].p,
        (uint64_t)(uintptr_t)h->Q[1].p, (uint64_t)(uintptr_t)h->H[0].p,
        (uint64_t)(uintptr_t)h->H[1].p, (uint64_t)(uintptr_t)h->Wb.p,
        (uint64_t)(uintptr_t)h->part.p, (uint64_t)(uintptr_t)h->Ysm.p,
        (uint64_t)(uintptr_t)h->Zsm.p, (uint64_t)(uintptr_t)h->hz.p,
        (uint64_t)(uintptr_t)h->Gs.p, (uint64_t)(uintptr_t)h->Rinv.p,
        (uint64_t)(uintptr_t)h->R1.p, (uint64_t)(uintptr_t)h->mask.p,
        (uint64_t)(uintptr_t)h->flags.p, (uint64_t)(uintptr_t)h->CM.p,
        (uint64_t)(uintptr_t)h->P.p, (uint64_t)(uintptr_t)h->PQ[0].p,
        (uint64_t)(uintptr_t)h->PQ[1].p, (uint64_t)S.track};
    uint64_t sig = 1469598103934665603ull;  // FNV-1a over the words
    for (uint64_t w : parts)
      for (int q = 0; q < 8; ++q) sig = (sig ^ ((w >> (8 * q)) & 0xff)) * 1099511628211ull;
    if (sig != h->graph_sig) {
      release_graphs(h);
      h->graph_sig = sig;
    }
  }

  hipEvent_t e0, e1, e2;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventCreate(&e2));
  HIPCHK(hipEventRecord(e0, h->stream));
  hipStream_t s = h->stream;
  h->op_used = 0;
  const int64_t nvec = std::min<int64_t>(S.kk, mmax);
  std::vector<double> theta(S.kk + 8), est(S.kk + 8);
  int64_t m = 0;
  int64_t iters = 0, restarts = 0;
  bool kconv = false;
  int flags_out = 0;
  if (t > h->k - 1) flags_out |= EDA_WARN_DEGENERATE;
  double bytes = 0.0;
  int64_t ops = 0;
  const double opbytes = 2.0 * d * h->N * dsize(h->storage) + 3.0 * d * b * qs;
  int64_t m_rr = 0;
  auto finite_pairs = [&](int64_t cnt) {
    for (int64_t i = 0; i < cnt; ++i)
      if (!std::isfinite(theta[i]) || !std::isfinite(est[i])) return false;
    return true;
  };
  // largest ratio residual / tolerance over the wanted pairs (<= 1: done)
  auto worst_ratio = [&]() {
    double w = 0.0;
    const double th1 = theta[0];
    for (int64_t i = 0; i < t; ++i) {
      const double thi = theta[i];
      if (!(thi > 0.0)) return (double)INFINITY;
      const double tol_i = std::max(tol, 10.0 * u_lo * th1 / thi);
      const double r = (o.resmode == EDA_RES_REL_THETA) ? est[i] / thi : est[i] / th1;
      if (!(r <= INFINITY)) return (double)INFINITY;
      w = std::max(w, r / tol_i);
    }
    return w;
  };
  auto phase_converged = [&]() { return worst_ratio() <= 1.0; };
  // Check schedule without a fixed interval: after two checks, the ratio's
  // decrease per block step predicts how many steps remain; the next check
  // comes after that many (at least 1, at most 4), else after 2.
  int64_t next_check = 0, prev_iter = -1;
  double prev_ratio = -1.0;
  auto schedule = [&](int64_t at_iter) {
    const double w = worst_ratio();
    int64_t gap = 2;
    if (prev_ratio > 0.0 && w < prev_ratio && at_iter > prev_iter && std::isfinite(w)) {
      const double rho = std::pow(w / prev_ratio, 1.0 / (double)(at_iter - prev_iter));
      if (rho > 0.0 && rho < 1.0) {
        const double k = std::ceil(std::log(w) / -std::log(rho));
        gap = (int64_t)std::max(1.0, std::min(4.0, k));
      }
    }
    prev_ratio = w;
    prev_iter = at_iter;
    next_check = at_iter + gap;
  };
  auto check_due = [&](bool can_check) {
    if (!can_check) return false;
    if (check_every > 0) return iters % check_every == 0;
    return iters >= next_check;
  };
  // Checks that need no restart run on the second stream, overlapping the
  // next block steps; the verdict is read when the next check is due (or
  // earlier, once ready).  A convergence found that way discards the steps
  // taken meanwhile.  EDA_SYNC_CHECKS=1 keeps every check synchronous.
  const bool async_checks = std::getenv("EDA_SYNC_CHECKS") == nullptr;
  if (async_checks) {
    if (h->aux == nullptr) HIPCHK(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    if (h->ev_main == nullptr) HIPCHK(hipEventCreateWithFlags(&h->ev_main, hipEventDisableTiming));
    if (h->ev_rr == nullptr) HIPCHK(hipEventCreateWithFlags(&h->ev_rr, hipEventDisableTiming));
    const size_t need = (size_t)2 * (S.kk + 8) * 8;
    if (h->rr_pin_cap < need) {
      if (h->rr_pin != nullptr) (void)hipHostFree(h->rr_pin);
      h->rr_pin = nullptr;
      h->rr_pin_cap = 0;
      if (hipHostMalloc((void**)&h->rr_pin, need, hipHostMallocDefault) != hipSuccess)
        return fail(h, EDA_ERR_NOMEM, "pinned readback allocation failed");
      h->rr_pin_cap = need;
    }
  }
  bool pending = false;
  int64_t pend_m = 0, pend_iter = 0;

  // ---- Krylov phase -------------------------------------------------------
  // The repair pass (second re-orthogonalisation of a new block) is needed
  // only when a block loses rank or most of its norm in the projection, which
  // happens as the Krylov space nears its dimension bound rank(P) + b <=
  // n - 1 + b.  Away from it the repair launches are left out; a flag raised
  // there anyway lands in a sticky slot, is seen at the next check, and the
  // Krylov phase is started again with the repair pass in every step.
  const int64_t sat = h->n - 1 + b;
  bool safe = std::getenv("EDA_ALWAYS_REPAIR") != nullptr;
  for (int attempt = 0;; ++attempt) {
  if (attempt > 0) {
    m = 0;
    iters = 0;
    restarts = 0;
    m_rr = 0;
    kconv = false;
    h->op_used = 0;
    next_check = 0;
    prev_iter = -1;
    prev_ratio = -1.0;
  }
    HIPCHK(launch_fill_i32(16, 0, h->flags.i(), s));
    HIPCHK(launch_fill(ldh * ldh, 0.0, h->H[0].d(), s));
    HIPCHK(launch_fill(ldh * ldh, 0.0, h->H[1].d(), s));
    S.cur = 0;

    // start block -> Q[:, 0:b] (drawn in float64, then cast to the basis type)
    void* Wst = h->Wb.p;
    double* Wst64 = h->Yb.d();
    if (o.start_block != nullptr)
      HIPCHK(launch_copy2d(d, b, o.start_block, DT::F64, o.ld_start, Wst, qdt, ldq, s));
    else {
      HIPCHK(launch_randn(d, b, o.seed, Wst64, ldq, s));
      HIPCHK(launch_copy2d(d, b, Wst64, DT::F64, ldq, Wst, qdt, ldq, s));
    }
    if (qdt == DT::F64)
      HIPCHK(launch_fill(ldq * (mmax + b), 0.0, (double*)S.Q(), s));
    else  // float32 zero has the bit pattern of int32 zero
      HIPCHK(launch_fill_i32(ldq * (mmax + b), 0, (int*)S.Q(), s));
    STCHK(cholqr_pass(h, d, b, Wst, qdt, ldq, S.Q(), ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                      nullptr, nullptr));
    STCHK(cholqr_pass(h, d, b, S.Q(), qdt, ldq, S.Q(), ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                      nullptr, nullptr));
  bool redo = false;
  while (true) {
    const bool repair = safe || (m + 3 * b >= sat);
    STCHK(lanczos_step(S, m, use_graphs, repair));
    m += b;
    ++iters;
    ops += b;
    bytes += opbytes;
    const bool need_restart = (m + b > mmax);
    const bool can_check = (m >= t + b) || need_restart;
    const bool due = check_due(can_check) || need_restart || iters >= max_iter;
    const bool must_sync = need_restart || iters >= max_iter;
    if (pending && (due || must_sync || hipEventQuery(h->ev_rr) == hipSuccess)) {
      int f2 = 0;
      STCHK(rr_collect(S, pend_m, t, theta.data(), est.data(), &f2));
      pending = false;
      m_rr = pend_m;
      if (f2 != 0 && !safe) { redo = true; break; }
      if (!finite_pairs(t)) return fail(h, EDA_ERR_NONFINITE, "non-finite Ritz pair in the Krylov phase");
      if (phase_converged()) {
        kconv = true;
        m = pend_m;  // the steps since then are not needed
        break;
      }
      schedule(pend_iter);
    }
    const bool due_now = check_due(can_check) || (can_check && must_sync);
    if (due_now && async_checks && !must_sync) {
      STCHK(rr_launch_async(S, m, std::min<int64_t>(t, m), t));
      pending = true;
      pend_m = m;
      pend_iter = iters;
      if (check_every == 0) next_check = iters + 2;  // refined when the verdict is read
    } else if (due_now) {
      // a restart keeps kk Ritz vectors in the basis: those must be
      // orthonormal (default cluster tolerance); a plain check needs t
      const int64_t cnt = need_restart ? S.kk : t;
      int f2 = 0;
      STCHK(rayleigh_ritz(S, m, std::min<int64_t>(need_restart ? nvec : t, m), cnt, theta.data(),
                          est.data(), &f2, need_restart ? 0.0 : kCheckCtol));
      m_rr = m;
      if (f2 != 0 && !safe) { redo = true; break; }
      if (!finite_pairs(cnt)) return fail(h, EDA_ERR_NONFINITE, "non-finite Ritz pair in the Krylov phase");
      if (phase_converged()) { kconv = true; break; }
      schedule(iters);
      if (iters >= max_iter) break;
      if (need_restart) {
        // thick restart: keep the kk leading Ritz vectors and the next block
        const int64_t kk = S.kk;
        HIPCHK(launch_gather_desc(m, kk, h->S.d(), mmax, h->Sd.d(), kk, s));
        const int nxt = 1 - S.cur;
        char* Qn = h->Q[nxt].c();
        double* Hn = h->H[nxt].d();
        HIPCHK(launch_nn(d, m, kk, S.Q(), qdt, ldq, h->Sd.d(), kk, 0.0, nullptr, qdt, ldq, Qn, qdt,
                         ldq, nullptr, s));
        HIPCHK(launch_copy2d(d, b, S.Qc(m), qdt, ldq, Qn + (size_t)kk * ldq * qs, qdt, ldq, s));
        // P^T of the kept Ritz vectors: (P^T Q) S_kk, row-major (the next
        // product fills the columns of the residual block)
        if (S.track)
          HIPCHK(launch_gemm(false, false, kk, h->N, m, 1.0, h->Sd.d(), kk, nullptr,
                             h->PQ[S.cur].d(), S.ldpq, 0.0, h->PQ[nxt].d(), S.ldpq, s));
        HIPCHK(launch_fill(ldh * ldh, 0.0, Hn, s));
        HIPCHK(launch_set_diag(kk, h->dtheta.d(), Hn, ldh, s));
        HIPCHK(launch_restart_coupling(m, b, kk, S.H() + m + (m - b) * ldh, ldh, h->Sd.d(), kk, Hn,
                                       ldh, s));
        S.cur = nxt;
        m = kk;
        ++restarts;
      }
    } else if (iters >= max_iter) {
      int f2 = 0;
      STCHK(rayleigh_ritz(S, m, std::min<int64_t>(t, m), std::min<int64_t>(t, m), theta.data(),
                          est.data(), &f2, kCheckCtol));
      m_rr = m;
      if (f2 != 0 && !safe) { redo = true; break; }
      break;
    }
  }
  if (!redo) break;
  if (pending) {  // drain the second stream before the buffers are reused
    HIPCHK(hipEventSynchronize(h->ev_rr));
    pending = false;
  }
  safe = true;
  }
  if (m_rr != m || m < t) {
    if (m < t) return fail(h, EDA_ERR_NOCONV, "basis smaller than t at the iteration limit");
    STCHK(rayleigh_ritz(S, m, std::min<int64_t>(t, m), t, theta.data(), est.data(), nullptr,
                        kCheckCtol));
  }

  // Ritz vectors Y = Q S_t in float64 (theta in dtheta)
  const size_t rw = (size_t)ldq * 2 * t;
  double* XB[2] = {h->refine.d(), h->refine.d() + rw};
  double* MB[2] = {h->refine.d() + 2 * rw, h->refine.d() + 3 * rw};
  int cb = 0;
  HIPCHK(launch_gather_desc(m, t, h->S.d(), mmax, h->Sd.d(), t, s));
  HIPCHK(launch_nn(d, m, t, S.Q(), qdt, ldq, h->Sd.d(), t, 0.0, nullptr, DT::F64, ldq, XB[0],
                   DT::F64, ldq, nullptr, s));
  HIPCHK(hipEventRecord(e1, s));

  // ---- float64 stage --------------------------------------------------------
  const double opbytes_t = 2.0 * d * h->N * 8.0 + 3.0 * d * t * 8.0;
  if (mixed && max_refine >= 0) {
    // orthonormalise the Ritz block in float64, apply the float64 operator
    // and take the Rayleigh-Ritz pairs of span(Y)
    STCHK(cholqr_pass(h, d, t, XB[0], DT::F64, ldq, h->Yb.d(), ldq, nullptr, nullptr, 0, nullptr,
                      0, 0, nullptr, nullptr));
    STCHK(cholqr_pass(h, d, t, h->Yb.d(), DT::F64, ldq, XB[0], ldq, nullptr, nullptr, 0, nullptr,
                      0, 0, nullptr, nullptr));
    STCHK(expop(h, true, 0, h->N, h->CM.d(), h->N, h->alphaB, t, XB[0], DT::F64, ldq, MB[0],
                DT::F64, ldq));
    ops += t;
    bytes += opbytes_t;
    STCHK(rr_block(h, d, ldq, t, t, mm, XB[0], MB[0], XB[1], MB[1]));
    cb = 1;
  } else if (S.track) {
    // P^T Y = (P^T Q) S_t (row-major N x t), then the second pass only
    HIPCHK(launch_gemm(false, false, t, h->N, m, 1.0, h->Sd.d(), t, nullptr, h->PQ[S.cur].d(),
                       S.ldpq, 0.0, h->Ysm.d(), t, s));
    STCHK(expop_second(h, true, 0, h->N, h->CM.d(), h->N, h->alphaB, t, XB[0], DT::F64, ldq,
                       MB[0], DT::F64, ldq));
    ops += t;
    bytes += opbytes_t;
  } else {
    STCHK(expop(h, true, 0, h->N, h->CM.d(), h->N, h->alphaB, t, XB[0], DT::F64, ldq, MB[0],
                DT::F64, ldq));
    ops += t;
    bytes += opbytes_t;
  }
  // h->Ysm holds P^T y for these Ritz vectors until the next product
  const double* ysm_of = (mixed && max_refine >= 0) ? nullptr : XB[0];
  std::vector<double> res(t);
  bool converged = false, floor_limited = false;
  int64_t passes = 0;
  // After a float64 Krylov phase the first explicit check nearly always
  // passes: the back-transform of the Ritz block is then enqueued before the
  // host reads the residuals, so the stream does not wait on the host (it is
  // redone for the refined block otherwise).
  const bool speculate = !mixed || max_refine < 0;
  bool x_done = false;
  int fl[2] = {0, 0};
  while (true) {
    double* Y = XB[cb];
    double* MY = MB[cb];
    double* Z = Y + (size_t)t * ldq;
    HIPCHK(launch_ritz_residual(d, t, MY, ldq, Y, ldq, h->dtheta.d(), Z, ldq, h->dres.d(), s));
    HIPCHK(hipEventRecord(e2, s));
    HIPCHK(hipMemcpyAsync(theta.data(), h->dtheta.d(), t * 8, hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(res.data(), h->dres.d(), t * 8, hipMemcpyDeviceToHost, s));
    x_done = false;
    if (speculate) {
      // x = exp(-S_W/2) y, orthonormalised in decreasing-lambda order
      // (Cholesky QR, twice), signs fixed
      STCHK(back_transform(h, t, Y, ldq, X, ldx, ldq, Y == ysm_of));
      x_done = true;
    }
    HIPCHK(hipMemcpyAsync(fl, h->flags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (std::getenv("EDA_LOG") != nullptr) log_pairs("f64", passes, t, theta.data(), res.data());
    bool ok = true;
    floor_limited = false;
    std::vector<int64_t> miss;  // pairs that miss their target
    const double th1 = theta[0];
    for (int64_t i = 0; i < t; ++i) {
      const double thi = theta[i];
      if (!(thi > 0.0)) { ok = false; miss.push_back(i); continue; }
      const double floor_i = 10.0 * kU64 * th1 / thi;
      if (floor_i > tol) floor_limited = true;
      const double r = (o.resmode == EDA_RES_REL_THETA) ? res[i] / thi : res[i] / th1;
      if (!(r <= std::max(tol, floor_i))) { ok = false; miss.push_back(i); }
    }
    if (ok) { converged = true; break; }
    if (!kconv || passes >= max_refine) break;
    // expand with the residuals of the pairs that miss their target: the
    // others are locked (span[Y, Z] contains their Ritz vectors, so
    // Rayleigh-Ritz keeps them), which keeps later passes narrow.
    // Z = orth(R) against Y and itself
    double* Zt = h->Yb.d();
    int64_t wzp = wz;
    if ((int64_t)miss.size() <= wz) {
      wzp = (int64_t)miss.size();
      // in ascending order: column miss[q] >= q is read before anything
      // overwrites it
      for (int64_t q = 0; q < wzp; ++q)
        if (miss[q] != q)
          HIPCHK(launch_copy2d(d, 1, Z + (size_t)miss[q] * ldq, DT::F64, ldq, Z + (size_t)q * ldq,
                               DT::F64, ldq, s));
    } else if (wz < t) {  // 2t > d: keep the residuals of the last (least converged) wz pairs
      HIPCHK(launch_copy2d(d, wz, Z + (size_t)(t - wz) * ldq, DT::F64, ldq, Zt, DT::F64, ldq, s));
      HIPCHK(launch_copy2d(d, wz, Zt, DT::F64, ldq, Z, DT::F64, ldq, s));
    }
    STCHK(cgs_pass(h, d, t, Y, DT::F64, ldq, Z, ldq, wzp, nullptr, 0, 0.0, nullptr));
    STCHK(cgs_pass(h, d, t, Y, DT::F64, ldq, Z, ldq, wzp, nullptr, 0, 0.0, nullptr));
    if (wzp <= 64) {
      // rank revealing on unit-norm columns: converged pairs leave columns of
      // roundoff; those are replaced by random directions
      const int64_t chunks = tn_chunks(d, wzp, wzp);
      HIPCHK(launch_tn_partial(d, wzp, wzp, Z, DT::F64, ldq, Z, DT::F64, ldq, h->part.d(), chunks,
                               nullptr, s));
      const bool fused = wzp <= 16;
      if (!fused)
        HIPCHK(launch_reduce_partials(chunks, wzp, wzp, h->part.d(), 1.0, 0.0, h->Gs.d(), wzp, 0.0,
                                      nullptr, 0, nullptr, s));
      HIPCHK(launch_pchol(wzp, h->Gs.d(), wzp, nullptr, 0, 0, 1e-10, 1e-4, true, h->Rinv.d(), wzp,
                          h->R1.d(), wzp, h->mask.i(), nullptr, s, fused ? h->part.d() : nullptr,
                          chunks));
      HIPCHK(launch_nn(d, wzp, wzp, Z, DT::F64, ldq, h->Rinv.d(), wzp, 0.0, nullptr, DT::F64, ldq, Zt,
                       DT::F64, ldq, nullptr, s, false, nullptr, nullptr, h->mask.i(),
                       0x7e41e000ull + (uint64_t)passes));
      STCHK(cgs_pass(h, d, t, Y, DT::F64, ldq, Zt, ldq, wzp, nullptr, 0, 0.0, nullptr));
      STCHK(cgs_pass(h, d, t, Y, DT::F64, ldq, Zt, ldq, wzp, nullptr, 0, 0.0, nullptr));
      STCHK(cholqr_pass(h, d, wzp, Zt, DT::F64, ldq, Z, ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                        nullptr, nullptr));
    } else {
      STCHK(cholqr_pass(h, d, wzp, Z, DT::F64, ldq, Zt, ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                        nullptr, nullptr));
      STCHK(cgs_pass(h, d, t, Y, DT::F64, ldq, Zt, ldq, wzp, nullptr, 0, 0.0, nullptr));
      STCHK(cholqr_pass(h, d, wzp, Zt, DT::F64, ldq, Z, ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                        nullptr, nullptr));
    }
    STCHK(cholqr_pass(h, d, wzp, Z, DT::F64, ldq, Zt, ldq, nullptr, nullptr, 0, nullptr, 0, 0,
                      nullptr, nullptr));
    HIPCHK(launch_copy2d(d, wzp, Zt, DT::F64, ldq, Z, DT::F64, ldq, s));
    STCHK(expop(h, true, 0, h->N, h->CM.d(), h->N, h->alphaB, wzp, Z, DT::F64, ldq,
                MY + (size_t)t * ldq, DT::F64, ldq));
    ysm_of = nullptr;
    ops += wzp;
    bytes += 2.0 * d * h->N * 8.0 + 3.0 * d * wzp * 8.0;
    STCHK(rr_block(h, d, ldq, t + wzp, t, mm, Y, MY, XB[1 - cb], MB[1 - cb]));
    cb = 1 - cb;
    ++passes;
  }
  if (!x_done) {
    // back-transform x = exp(-S_W/2) y, orthonormalise in decreasing-lambda
    // order (Cholesky QR, twice), then fix signs
    STCHK(back_transform(h, t, XB[cb], ldq, X, ldx, ldq));
    HIPCHK(hipMemcpyAsync(fl, h->flags.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  float kms = 0.f, rms = 0.f;
  HIPCHK(hipEventElapsedTime(&kms, e0, e1));
  HIPCHK(hipEventElapsedTime(&rms, e1, e2));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipEventDestroy(e2);

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
  if (floor_limited) flags_out |= EDA_WARN_FLOOR;
  if (fl[1] | fl[0]) flags_out |= EDA_WARN_REPAIRED;
  if (info != nullptr) {
    info->iters = (int32_t)iters;
    info->restarts = (int32_t)restarts;
    info->refine_passes = (int32_t)passes;
    info->flags = flags_out;
    info->ops = ops;
    info->bytes_moved = bytes;
    info->t_prepare_ms = prepare_time_ms(h);
    info->t_krylov_ms = kms;
    info->t_refine_ms = rms;
    info->shift_s = h->shiftB;
    double top = 0.0;
    for (size_t q = 0; q + 1 < h->op_used; q += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, h->op_ev[q], h->op_ev[q + 1]) == hipSuccess) top += ms;
    }
    info->op_calls = (int64_t)(h->op_used / 2);
    info->t_op_ms = top;
    info->op_bytes = opbytes;
  }
  if (range_err) return fail(h, EDA_ERR_RANGE, "a Ritz value underflowed after the shift");
  if (!converged) {
    if (!kconv) return fail(h, EDA_ERR_NOCONV, "max_iter reached before convergence");
    return fail(h, EDA_ERR_NOCONV, "float64 refinement did not reach the tolerance in %lld passes",
                (long long)passes);
  }
  return EDA_OK;
}
