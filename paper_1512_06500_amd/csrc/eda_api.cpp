// libeda host library, part 1: handle, validation, preprocessing (factor
// ingest, Gram, small eigensolves, cores) and the exponential products.
// Every numerical step runs in the kernels of this directory; the host only
// validates, allocates, orders launches on the handle's stream and takes the
// small scalar decisions (spectral shift, scaling of the polynomial).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "host_internal.h"

using namespace eda;

namespace eda {

eda_status fail(eda_handle h, eda_status s, const char* fmt, ...) {
  if (h != nullptr) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    h->err = buf;
  }
  return s;
}

eda_status ensure(eda_handle h, Buf& b, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (b.cap >= bytes) return EDA_OK;
  if (b.p != nullptr) {
    HIPCHK(hipStreamSynchronize(h->stream));
    HIPCHK(hipFree(b.p));
    b.p = nullptr;
    b.cap = 0;
  }
  size_t rounded = ((bytes + 4095) / 4096) * 4096;
  if (hipMalloc(&b.p, rounded) != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(h, EDA_ERR_NOMEM, "device allocation of %zu bytes failed", rounded);
  }
  b.cap = rounded;
  return EDA_OK;
}

void release(Buf& b) {
  if (b.p != nullptr) (void)hipFree(b.p);
  b.p = nullptr;
  b.cap = 0;
}

eda_status need_device(eda_handle h) {
  if (h->device < 0) return fail(h, EDA_ERR_HIP, "no HIP device available to this handle");
  return EDA_OK;
}

eda_status check_dev_ptr(eda_handle h, const void* p, const char* name) {
  hipPointerAttribute_t attr;
  hipError_t e = hipPointerGetAttributes(&attr, p);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return fail(h, EDA_ERR_ARG, "%s is not a device pointer", name);
  }
  if (attr.type != hipMemoryTypeDevice && attr.type != hipMemoryTypeManaged &&
      attr.type != hipMemoryTypeUnified)
    return fail(h, EDA_ERR_ARG, "%s is not device memory", name);
  return EDA_OK;
}

// Low-rank exponential apply on columns [c0, c0+Nc) of P:
//   Out = alpha V + P_c (C (P_c^T V)),  C: Nc x Nc (ldc).
namespace {
const char* p_columns(eda_handle h, bool master, int64_t c0, DT* pdt) {
  const bool use64 = master && h->storage != EDA_F64;
  *pdt = use64 ? DT::F64 : dt_of(h->storage);
  const char* base = use64 ? h->P64.c() : h->P.c();
  return base + (size_t)c0 * h->ldp * dt_size(*pdt);
}
}  // namespace

eda_status expop_first(eda_handle h, bool master, int64_t c0, int64_t Nc, int64_t b,
                       const void* V, DT vdt, int64_t ldv, double* ysm, int64_t ldy) {
  DT pdt;
  const char* Pc = p_columns(h, master, c0, &pdt);
  const int64_t chunks = tn_chunks(h->d, Nc, b);
  STCHK(ensure(h, h->part, (size_t)chunks * Nc * b * 8));
  if (ysm == nullptr) {
    STCHK(ensure(h, h->Ysm, (size_t)Nc * b * 8));
    ysm = h->Ysm.d();
    ldy = b;
  }
  const double* sc = (pdt == DT::FP8) ? h->pscale.d() + c0 : nullptr;
  HIPCHK(launch_tn_partial(h->d, Nc, b, Pc, pdt, h->ldp, V, vdt, ldv, h->part.d(), chunks,
                           nullptr, h->stream, sc));
  // Y = P_c^T V (row-major)
  HIPCHK(launch_reduce_partials(chunks, Nc, b, h->part.d(), 0.0, 0.0, nullptr, 0, 1.0, ysm, ldy,
                                nullptr, h->stream));
  return EDA_OK;
}

eda_status expop_second(eda_handle h, bool master, int64_t c0, int64_t Nc, const double* C,
                        int64_t ldc, double alpha, int64_t b, const void* V, DT vdt,
                        int64_t ldv, void* Out, DT odt, int64_t ldo, const double* alpha_p,
                        const double* ysm, int64_t ldy) {
  DT pdt;
  const char* Pc = p_columns(h, master, c0, &pdt);
  STCHK(ensure(h, h->Zsm, (size_t)Nc * b * 8));
  if (ysm == nullptr) {
    ysm = h->Ysm.d();
    ldy = b;
  }
  const double* sc = (pdt == DT::FP8) ? h->pscale.d() + c0 : nullptr;
  // Z = C Y (row-major) by the same streaming kernel with C as the tall
  // operand (split over column groups of C when it is large), then
  // Out = alpha V + P_c Z
  bool done = false;
  if (core_split(Nc, b, C, ldc)) {
    STCHK(ensure(h, h->zpart, (size_t)nn_split_groups(Nc) * Nc * b * 8));
    HIPCHK(launch_nn_split(Nc, b, C, ldc, ysm, ldy, h->zpart.d(), h->Zsm.d(), b, h->stream));
    done = true;
  } else if (b > 16 && Nc >= 256) {
    // a wide block (Ritz blocks of the final stage): Z^T = Y^T C^T on the
    // matrix cores, Y^T and Z^T being the row-major Y and Z read column-major
    HIPCHK(launch_gemm(false, true, b, Nc, Nc, 1.0, ysm, ldy, nullptr, C, ldc, 0.0, h->Zsm.d(), b,
                       h->stream));
    done = true;
  }
  if (!done)
    HIPCHK(launch_nn(Nc, Nc, b, C, DT::F64, ldc, ysm, ldy, 0.0, nullptr, DT::F64, 0, h->Zsm.d(),
                     DT::F64, b, nullptr, h->stream, true));
  if (narrow_split(pdt, vdt, odt, b, h->ldp)) {
    // narrow factor and block: column groups of P, float32 partial rows,
    // fixed-order sum (a float64 block keeps float64 sums below)
    STCHK(ensure(h, h->npart, (size_t)nn_narrow_split_groups(h->d, Nc) * h->d * 8 * 4));
    const hipError_t e = launch_nn_narrow_split(h->d, Nc, b, Pc, pdt, h->ldp, h->Zsm.d(), b, alpha,
                                                alpha_p, V, vdt, ldv, Out, odt, ldo, sc,
                                                (float*)h->npart.p, h->stream);
    if (e == hipSuccess) return EDA_OK;
    if (e != hipErrorInvalidValue)
      return fail(h, EDA_ERR_HIP, "launch_nn_narrow_split failed: %s", hipGetErrorString(e));
  }
  HIPCHK(launch_nn(h->d, Nc, b, Pc, pdt, h->ldp, h->Zsm.d(), b, alpha, V, vdt, ldv, Out, odt,
                   ldo, nullptr, h->stream, false, alpha_p, sc));
  return EDA_OK;
}

eda_status expop(eda_handle h, bool master, int64_t c0, int64_t Nc, const double* C,
                 int64_t ldc, double alpha, int64_t b, const void* V, DT vdt, int64_t ldv,
                 void* Out, DT odt, int64_t ldo, const double* alpha_p) {
  STCHK(expop_first(h, master, c0, Nc, b, V, vdt, ldv));
  return expop_second(h, master, c0, Nc, C, ldc, alpha, b, V, vdt, ldv, Out, odt, ldo, alpha_p);
}

}  // namespace eda

namespace {

// launch_gemm_sym on the handle's stream with the handle's split workspace
eda_status gemm_sym(eda_handle h, bool ta, bool tb, int64_t n, int64_t k, double alpha,
                    const double* A, int64_t lda, const double* dk, const double* B, int64_t ldb,
                    double beta, double* C, int64_t ldc) {
  const int64_t wsb = gemm_sym_ws_bytes(n, k);
  if (wsb > 0) STCHK(ensure(h, h->gws, (size_t)wsb));
  HIPCHK(launch_gemm_sym(ta, tb, n, k, alpha, A, lda, dk, B, ldb, beta, C, ldc, h->stream,
                         wsb > 0 ? h->gws.d() : nullptr, wsb));
  return EDA_OK;
}

// Core V diag(f) V^T of exp(c H H^T) e^{-shift} for the factor `which`.
// W-core by a matrix polynomial instead of an eigendecomposition:
//   G_c = c psi(c G_WW),  psi(X) = sum_{j>=0} X^j / (j+1)!  (psi(z) = (e^z - 1)/z),
// which equals V diag(phi_c(lambda)) V^T.  X = c G_WW has its spectrum in
// [-rho, 0] (c <= 0), and rho <= ||X^p||_1^{1/p} for every p, so the 1-norms
// of X, X^2 and X^4 (the last two are powers the evaluation needs anyway)
// bound it (X alone where the host must not wait for the device); with the
// scale f = 2^-q that brings the bound to at most 2,
// psi(f X) is the Taylor polynomial of degree 23 (alternating remainder
// below 2^24 / 25! < 1.1e-18, terms at most 1 against psi(-2) = 0.43),
// evaluated by Paterson-Stockmeyer on the powers of X with the powers of f
// folded into the coefficients, then q doublings
// psi(2Y) = psi(Y) + psi(Y) Y psi(Y) / 2.  Only GEMMs.
eda_status poly_core_W(eda_handle h, double c, double* out) {
  const int64_t n = h->n, N = h->N, nn = n * n;
  hipStream_t s = h->stream;
  STCHK(ensure(h, h->polyws, (size_t)7 * nn * 8));
  STCHK(ensure(h, h->normbuf, 64));
  double* X = h->polyws.d();
  double* A2 = X + nn;
  double* A3 = A2 + nn;
  double* A4 = A3 + nn;
  double* P = A4 + nn;
  double* T = P + nn;
  double* U = T + nn;
  constexpr int kDeg = 23;            // degree of the Taylor polynomial
  constexpr int kChunks = (kDeg + 1) / 4;
  double a[kDeg + 1];
  double fct = 1.0;
  for (int j = 0; j <= kDeg; ++j) {
    fct *= (double)(j + 1);
    a[j] = 1.0 / fct;  // 1/(j+1)!
  }
  // every product below is of commuting symmetric polynomials in X, hence
  // symmetric: only lower triangles are computed (and mirrored)
  HIPCHK(launch_copy_block(n, n, c, h->G.d(), N, false, X, n, s));
  STCHK(gemm_sym(h, false, false, n, n, 1.0, X, n, nullptr, X, n, 0.0, A2, n));
  STCHK(gemm_sym(h, false, false, n, n, 1.0, A2, n, nullptr, A2, n, 0.0, A4, n));
  double rho = std::fabs(c) * h->normW;
  if (h->poly_readback) {
    HIPCHK(launch_norm1(n, A2, n, h->normbuf.d() + 1, s));
    HIPCHK(launch_norm1(n, A4, n, h->normbuf.d() + 2, s));
    double nrm[2] = {0.0, 0.0};
    HIPCHK(hipMemcpyAsync(nrm, h->normbuf.d() + 1, sizeof(nrm), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (std::isfinite(nrm[0])) rho = std::min(rho, std::sqrt(nrm[0]));
    if (std::isfinite(nrm[1])) rho = std::min(rho, std::sqrt(std::sqrt(nrm[1])));
  }
  int q = 0;
  while (rho > 2.0 && q < 60) {
    rho *= 0.5;
    ++q;
  }
  const double f = std::ldexp(1.0, -q), f2 = f * f, f3 = f2 * f, f4 = f2 * f2;
  // A3 = (f X)^3; chunk k of the polynomial in Y = f X is
  // a_{4k} I + a_{4k+1} Y + a_{4k+2} Y^2 + a_{4k+3} Y^3, and P <- chunk + Y^4 P
  STCHK(gemm_sym(h, false, false, n, n, f3, A2, n, nullptr, X, n, 0.0, A3, n));
  int kb = kChunks - 1;
  HIPCHK(launch_lincomb(n, a[4 * kb], a[4 * kb + 1] * f, X, a[4 * kb + 2] * f2, A2,
                        a[4 * kb + 3], A3, n, P, n, s));
  for (kb = kChunks - 2; kb >= 0; --kb) {
    HIPCHK(launch_lincomb(n, a[4 * kb], a[4 * kb + 1] * f, X, a[4 * kb + 2] * f2, A2,
                          a[4 * kb + 3], A3, n, T, n, s));
    STCHK(gemm_sym(h, false, false, n, n, f4, A4, n, nullptr, P, n, 1.0, T, n));
    std::swap(P, T);
  }
  if (q > 0) HIPCHK(launch_copy_block(n, n, f, X, n, false, X, n, s));  // X <- Y
  for (int i = 0; i < q; ++i) {
    STCHK(gemm_sym(h, false, false, n, n, 1.0, X, n, nullptr, P, n, 0.0, U, n));
    HIPCHK(launch_copy_block(n, n, 1.0, P, n, false, T, n, s));
    STCHK(gemm_sym(h, false, false, n, n, 0.5, P, n, nullptr, U, n, 1.0, T, n));
    std::swap(P, T);
    HIPCHK(launch_copy_block(n, n, 2.0, X, n, false, X, n, s));
  }
  // symmetrise (rounding) and scale by c
  HIPCHK(launch_symmetrize(n, P, n, out, n, s));
  HIPCHK(launch_copy_block(n, n, c, out, n, false, out, n, s));
  return EDA_OK;
}

// Eigenpairs of H_W^T H_W on demand (the polynomial route does not need them).
eda_status ensure_w_eig(eda_handle h) {
  if (h->w_eig) return EDA_OK;
  const int64_t n = h->n;
  STCHK(ensure(h, h->syev_work, syev_work_bytes(n)));
  HIPCHK(launch_syev(1, n, nullptr, h->G.d(), h->N, 0, h->eigW.d(), 0, h->eigZ.d(), n, 0, 0,
                     h->syev_work.d(), h->stream));
  h->hwW.assign(n, 0.0);
  HIPCHK(hipMemcpyAsync(h->hwW.data(), h->eigW.d(), n * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  h->w_eig = true;
  return EDA_OK;
}

eda_status build_core(eda_handle h, int which, double c, double shift, double* out) {
  if (which == EDA_W && !h->w_eig) {
    if (c <= 0.0) return poly_core_W(h, c, out);
    STCHK(ensure_w_eig(h));
  }
  const int64_t Nw = which == EDA_W ? h->n : h->k;
  const double* lam = h->eigW.d() + (which == EDA_W ? 0 : h->n);
  const double* Z = h->eigZ.d() + (which == EDA_W ? 0 : h->n * h->n);
  const int64_t ldz = h->n;
  STCHK(ensure(h, h->fw, (size_t)(h->N + 8) * 8));
  HIPCHK(launch_core_weights(Nw, lam, c, shift, h->fw.d(), h->stream));
  STCHK(gemm_sym(h, false, true, Nw, Nw, 1.0, Z, ldz, h->fw.d(), Z, ldz, 0.0, out, Nw));
  return EDA_OK;
}

// G_h = phi_{-1/2}(H_W^T H_W) and G_m = phi_{-1}(H_W^T H_W).
eda_status build_w_cores(eda_handle h) {
  const int64_t n = h->n, N = h->N;
  STCHK(ensure(h, h->Gh, (size_t)n * n * 8));
  STCHK(ensure(h, h->Gm, (size_t)n * n * 8));
  STCHK(ensure(h, h->CM, (size_t)N * N * 8));
  STCHK(build_core(h, EDA_W, -0.5, 0.0, h->Gh.d()));
  if (h->w_eig) {
    STCHK(build_core(h, EDA_W, -1.0, 0.0, h->Gm.d()));
  } else {
    // exp(-S_W) = exp(-S_W/2)^2 gives G_m = 2 G_h + G_h (H_W^T H_W) G_h
    STCHK(gemm_sym(h, false, false, n, n, 1.0, h->G.d(), N, nullptr, h->Gh.d(), n, 0.0,
                       h->CM.d(), n));
    HIPCHK(launch_copy_block(n, n, 2.0, h->Gh.d(), n, false, h->Gm.d(), n, h->stream));
    STCHK(gemm_sym(h, false, false, n, n, 1.0, h->Gh.d(), n, nullptr, h->CM.d(), n, 1.0,
                       h->Gm.d(), n));
  }
  return EDA_OK;
}

// G_B = e^{-s} phi_1(H_B^T H_B) and the composite cores C_M, C_A (after the
// W-cores and the shift).
eda_status build_composite_cores(eda_handle h) {
  const int64_t n = h->n, k = h->k, N = h->N;
  STCHK(ensure(h, h->GBs, (size_t)k * k * 8));
  STCHK(ensure(h, h->CM, (size_t)N * N * 8));
  STCHK(ensure(h, h->T1, (size_t)n * k * 8));
  STCHK(ensure(h, h->T2, (size_t)n * k * 8));
  STCHK(build_core(h, EDA_B, 1.0, h->shiftB, h->GBs.d()));
  const double* K = h->G.d() + n * N;  // H_W^T H_B, n x k, ld N
  hipStream_t s = h->stream;
  double* CM = h->CM.d();
  h->ca_ready = false;
  // Lanczos core: [[a Gm + Gh K GB K^T Gh, Gh K GB], [GB K^T Gh, GB]]
  HIPCHK(launch_gemm(false, false, n, k, n, 1.0, h->Gh.d(), n, nullptr, K, N, 0.0, h->T1.d(), n, s));
  HIPCHK(launch_gemm(false, false, n, k, k, 1.0, h->T1.d(), n, nullptr, h->GBs.d(), k, 0.0,
                     h->T2.d(), n, s));
  HIPCHK(launch_copy_block(n, n, h->alphaB, h->Gm.d(), n, false, CM, N, s));
  HIPCHK(launch_gemm_sym(false, true, n, k, 1.0, h->T2.d(), n, nullptr, h->T1.d(), n, 1.0, CM, N, s));
  HIPCHK(launch_copy_block(n, k, 1.0, h->T2.d(), n, false, CM + n * N, N, s));
  HIPCHK(launch_copy_block(k, n, 1.0, h->T2.d(), n, true, CM + n, N, s));
  HIPCHK(launch_copy_block(k, k, 1.0, h->GBs.d(), k, false, CM + n + n * N, N, s));
  return EDA_OK;
}

}  // namespace

namespace eda {

// Arnoldi core: [[a Gm, Gm K GB], [0, GB]]
eda_status promote_storage_f64(eda_handle h) {
  if (!h->prepared) return fail(h, EDA_ERR_STATE, "no preparation to promote");
  if (h->storage == EDA_F64) return EDA_OK;
  std::swap(h->P, h->P64);
  release(h->P64);
  h->storage = EDA_F64;
  release_graphs(h);  // captured steps read the narrow copy
  return EDA_OK;
}

eda_status warm_start_block(eda_handle h, int64_t d, int64_t t, int64_t b, const double* Y,
                            int64_t ldy, uint64_t seed, double** V, int64_t* ldv) {
  STCHK(ensure(h, h->warm, (size_t)(d * b + t * b) * 8));
  double* Vd = h->warm.d();
  hipStream_t s = h->stream;
  if (t >= b) {
    // G: t x b with entries +-1 from a SplitMix64 stream (Steele, Lea and
    // Flood 2014), scaled by 1/sqrt(t); every column of Y G mixes all pairs
    std::vector<double> G((size_t)t * b);
    uint64_t x = seed ^ 0x243f6a8885a308d3ull;
    const double sc = 1.0 / std::sqrt((double)t);
    for (auto& g : G) {
      x += 0x9e3779b97f4a7c15ull;
      uint64_t z = x;
      z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
      z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
      z ^= z >> 31;
      g = (z >> 63) ? sc : -sc;
    }
    double* Gd = Vd + d * b;
    HIPCHK(hipMemcpyAsync(Gd, G.data(), G.size() * 8, hipMemcpyHostToDevice, s));
    HIPCHK(launch_gemm(false, false, d, b, t, 1.0, Y, ldy, nullptr, Gd, t, 0.0, Vd, d, s));
    HIPCHK(hipStreamSynchronize(s));  // G is a host temporary
  } else {
    HIPCHK(launch_copy2d(d, t, Y, DT::F64, ldy, Vd, DT::F64, d, s));
    HIPCHK(launch_randn(d, b - t, seed, Vd + d * t, d, s));
  }
  *V = Vd;
  *ldv = d;
  return EDA_OK;
}

eda_status ensure_arnoldi_core(eda_handle h) {
  if (h->ca_ready) return EDA_OK;
  const int64_t n = h->n, k = h->k, N = h->N;
  STCHK(ensure(h, h->CA, (size_t)N * N * 8));
  STCHK(ensure(h, h->T3, (size_t)n * k * 8));
  STCHK(ensure(h, h->T4, (size_t)n * k * 8));
  const double* K = h->G.d() + n * N;  // H_W^T H_B, n x k, ld N
  hipStream_t s = h->stream;
  double* CA = h->CA.d();
  HIPCHK(launch_gemm(false, false, n, k, n, 1.0, h->Gm.d(), n, nullptr, K, N, 0.0, h->T3.d(), n, s));
  HIPCHK(launch_gemm(false, false, n, k, k, 1.0, h->T3.d(), n, nullptr, h->GBs.d(), k, 0.0,
                     h->T4.d(), n, s));
  HIPCHK(launch_copy_block(n, n, h->alphaB, h->Gm.d(), n, false, CA, N, s));
  HIPCHK(launch_copy_block(n, k, 1.0, h->T4.d(), n, false, CA + n * N, N, s));
  HIPCHK(launch_copy_block(k, n, 0.0, h->T4.d(), n, true, CA + n, N, s));
  HIPCHK(launch_copy_block(k, k, 1.0, h->GBs.d(), k, false, CA + n + n * N, N, s));
  h->ca_ready = true;
  return EDA_OK;
}

}  // namespace eda

namespace eda {

eda_status validate_block(eda_handle h, int64_t b, const void* V, int64_t ldv, const void* Out,
                          int64_t ldo, eda_dtype vdtype) {
  if (b < 1 || b > (1 << 20)) return fail(h, EDA_ERR_ARG, "block width b=%lld out of range", (long long)b);
  if (V == nullptr || Out == nullptr) return fail(h, EDA_ERR_ARG, "null V or Out");
  if (vdtype != EDA_F64 && vdtype != EDA_F32 && vdtype != EDA_BF16)
    return fail(h, EDA_ERR_ARG, "vdtype must be EDA_F64, EDA_F32 or EDA_BF16");
  if (vdtype == EDA_BF16 && h->storage != EDA_BF16 && h->storage != EDA_FP8_E4M3)
    return fail(h, EDA_ERR_ARG, "a bfloat16 block needs bfloat16 or FP8 storage");
  if (ldv < h->d || ldo < h->d) return fail(h, EDA_ERR_ARG, "ldv/ldo must be >= d");
  const size_t es = dsize(vdtype);
  const char* v0 = (const char*)V;
  const char* v1 = v0 + ((b - 1) * ldv + h->d) * es;
  const char* o0 = (const char*)Out;
  const char* o1 = o0 + ((b - 1) * ldo + h->d) * es;
  if (v0 < o1 && o0 < v1) return fail(h, EDA_ERR_ARG, "V and Out overlap");
  return EDA_OK;
}

}  // namespace eda

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* eda_strerror(eda_status s) {
  switch (s) {
    case EDA_OK: return "success";
    case EDA_ERR_ARG: return "invalid argument";
    case EDA_ERR_NOMEM: return "out of memory";
    case EDA_ERR_HIP: return "HIP runtime error";
    case EDA_ERR_NOCONV: return "iteration limit reached before convergence";
    case EDA_ERR_RANGE: return "result out of floating-point range";
    case EDA_ERR_NONFINITE: return "non-finite value in input";
    case EDA_ERR_STATE: return "call order violated";
  }
  return "unknown status";
}

const char* eda_last_error(eda_handle h) {
  if (h == nullptr) return "null handle";
  return h->err.c_str();
}

eda_status eda_create(eda_handle* out, void* hip_stream) {
  if (out == nullptr) return EDA_ERR_ARG;
  eda_handle h = new (std::nothrow) eda_handle_s();
  if (h == nullptr) return EDA_ERR_NOMEM;
  *out = h;
  h->stream = (hipStream_t)hip_stream;
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) {
    (void)hipGetLastError();
    h->device = -1;
    return fail(h, EDA_ERR_HIP, "no HIP device: the handle can only validate arguments");
  }
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || count < 1) {
    (void)hipGetLastError();
    h->device = -1;
    return fail(h, EDA_ERR_HIP, "no HIP device: the handle can only validate arguments");
  }
  h->device = dev;
  if (std::getenv("EDA_SYEV_TIMERS") != nullptr) syev_timing_enable(true);
  // device address of the allocation-free entry point's scratch array on
  // this device (a failure is reported by that entry point, not here)
  (void)noalloc_init_device(dev);
  return EDA_OK;
}

void eda_destroy(eda_handle h) {
  if (h == nullptr) return;
  if (h->device >= 0 && std::getenv("EDA_SYEV_TIMERS") != nullptr) {
    (void)hipStreamSynchronize(h->stream);
    syev_timing_report(stderr);
  }
  if (h->device >= 0) {
    (void)hipStreamSynchronize(h->stream);
    Buf* all[] = {&h->polyws, &h->normbuf,
                  &h->P,  &h->G,  &h->eigW, &h->eigZ, &h->nsbuf, &h->Gh,  &h->Gm,  &h->GBs,
                  &h->CM, &h->CA, &h->T1,   &h->T2,   &h->T3,    &h->T4,  &h->fw,  &h->part, &h->zpart,
                  &h->Ysm, &h->Zsm, &h->PQ[0], &h->PQ[1], &h->syev_work, &h->offs, &h->flags, &h->mask, &h->Q[0], &h->Q[1],
                  &h->H[0], &h->H[1], &h->Wb, &h->T, &h->wT, &h->S, &h->Sd, &h->hz, &h->Gs,
                  &h->Rinv, &h->R1, &h->Yb, &h->MYb, &h->dtheta, &h->dres, &h->P64, &h->refine, &h->alphaB_dev, &h->pscale, &h->warm, &h->npart, &h->gws};
    for (Buf& b : h->dir) release(b);
    for (Buf& b : h->af) release(b);
    for (Buf& b : h->nnp) release(b);
    for (Buf* b : all) release(*b);
    for (auto& c : h->cores) release(c.buf);
    for (hipEvent_t e : h->op_ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : h->prep_ev)
      if (e != nullptr) (void)hipEventDestroy(e);
    if (h->pin != nullptr) (void)hipHostFree(h->pin);
    if (h->rr_pin != nullptr) (void)hipHostFree(h->rr_pin);
    if (h->ev_main != nullptr) (void)hipEventDestroy(h->ev_main);
    if (h->ev_rr != nullptr) (void)hipEventDestroy(h->ev_rr);
    if (h->aux != nullptr) (void)hipStreamDestroy(h->aux);
    release_graphs(h);
    if (h->cap != nullptr) (void)hipStreamDestroy(h->cap);
    destroy_batch_state(h);
  }
  delete h;
}

eda_status eda_scatter_factors(eda_handle h, int64_t d, int64_t n, int64_t k, const double* X,
                               int64_t ldx, const int64_t* counts, double* H_W, int64_t ldw,
                               double* H_B, int64_t ldb) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (d < 1 || n < 1 || k < 1 || k > n) return fail(h, EDA_ERR_ARG, "need d>=1, 1<=k<=n");
  if (k > 65535) return fail(h, EDA_ERR_ARG, "k=%lld exceeds 65535 classes", (long long)k);
  if (X == nullptr || counts == nullptr || H_W == nullptr || H_B == nullptr)
    return fail(h, EDA_ERR_ARG, "null pointer argument");
  if (ldx < d || ldw < d || ldb < d) return fail(h, EDA_ERR_ARG, "leading dimensions must be >= d");
  std::vector<int64_t> offs(k + 1, 0);
  for (int64_t j = 0; j < k; ++j) {
    if (counts[j] < 1) return fail(h, EDA_ERR_ARG, "class %lld has no samples", (long long)j);
    offs[j + 1] = offs[j] + counts[j];
  }
  if (offs[k] != n) return fail(h, EDA_ERR_ARG, "class sizes sum to %lld, not n=%lld",
                                (long long)offs[k], (long long)n);
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, X, "X"));
  STCHK(check_dev_ptr(h, H_W, "H_W"));
  STCHK(check_dev_ptr(h, H_B, "H_B"));
  STCHK(ensure(h, h->offs, (size_t)(k + 1) * 8));
  HIPCHK(hipMemcpyAsync(h->offs.p, offs.data(), (size_t)(k + 1) * 8, hipMemcpyHostToDevice,
                        h->stream));
  HIPCHK(launch_scatter(d, n, k, X, ldx, (const int64_t*)h->offs.p, H_W, ldw, H_B, ldb,
                        h->stream));
  // the host array must outlive the copy
  HIPCHK(hipStreamSynchronize(h->stream));
  return EDA_OK;
}

}  // extern "C"

namespace eda {

eda_status build_w_core(eda_handle h, double c, double* out) {
  if (c > 0.0) STCHK(ensure_w_eig(h));
  return build_core(h, EDA_W, c, 0.0, out);
}

void release_graphs(eda_handle h) {
  for (auto& g : h->graphs) {
    if (g.op != nullptr) (void)hipGraphExecDestroy(g.op);
    if (g.rest != nullptr) (void)hipGraphExecDestroy(g.rest);
  }
  h->graphs.clear();
  h->graph_sig = 0;
}

eda_status prepare_begin(eda_handle h, int64_t d, int64_t n, int64_t k, const double* H_W,
                         int64_t ldw, const double* H_B, int64_t ldb, eda_dtype storage,
                         bool overlap) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (d < 2 || k < 2 || n < k) return fail(h, EDA_ERR_ARG, "need d>=2, k>=2, n>=k");
  // the dense eigensolves of the preparation are of sizes k and (on request) n
  if (n > 2048) return fail(h, EDA_ERR_ARG, "n=%lld exceeds 2048", (long long)n);
  if (H_W == nullptr || H_B == nullptr) return fail(h, EDA_ERR_ARG, "null factor");
  if (ldw < d || ldb < d) return fail(h, EDA_ERR_ARG, "leading dimensions must be >= d");
  if (storage != EDA_F64 && storage != EDA_F32 && storage != EDA_BF16 && storage != EDA_FP8_E4M3)
    return fail(h, EDA_ERR_ARG, "storage must be EDA_F64, EDA_F32, EDA_BF16 or EDA_FP8_E4M3");
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, H_W, "H_W"));
  STCHK(check_dev_ptr(h, H_B, "H_B"));
  h->prepared = false;
  for (auto& c : h->cores) release(c.buf);
  h->cores.clear();

  for (int q = 0; q < 4; ++q)
    if (h->prep_ev[q] == nullptr) HIPCHK(hipEventCreate(&h->prep_ev[q]));
  (void)prepare_time_ms(h);
  HIPCHK(hipEventRecord(h->prep_ev[0], h->stream));

  const int64_t N = n + k;
  h->d = d;
  h->n = n;
  h->k = k;
  h->N = N;
  h->storage = storage;
  h->ldp = round_up(d, 64);

  // pinned scalars: [flag | normW | eig(G_BB) (k) | eig(G_WW) (n)]
  const size_t pin_bytes = (size_t)(2 + k + n) * 8;
  if (h->pin_cap < pin_bytes) {
    if (h->pin != nullptr) {
      HIPCHK(hipStreamSynchronize(h->stream));
      (void)hipHostFree(h->pin);
      h->pin = nullptr;
      h->pin_cap = 0;
    }
    if (hipHostMalloc(&h->pin, pin_bytes, hipHostMallocDefault) != hipSuccess) {
      (void)hipGetLastError();
      h->pin = nullptr;
      return fail(h, EDA_ERR_NOMEM, "pinned host allocation of %zu bytes failed", pin_bytes);
    }
    h->pin_cap = pin_bytes;
  }
  double* pin = (double*)h->pin;

  STCHK(ensure(h, h->flags, 64));
  HIPCHK(launch_fill_i32(16, 0, h->flags.i(), h->stream));

  // a1: factor ingest, P = [H_W H_B] in storage precision, plus a float64
  // master when the storage is narrower (Gram, cores and refinement use it)
  // (FP8: per-column scales from the master, then the scaled E4M3 copy).
  // The float64 copy also flags non-finite entries of the factors.
  int* nf = h->flags.i();
  STCHK(ensure(h, h->P, (size_t)h->ldp * N * dsize(storage)));
  if (storage != EDA_FP8_E4M3) {
    int* f = (storage == EDA_F64) ? nf : nullptr;
    HIPCHK(launch_pack(d, h->ldp, n, H_W, ldw, h->P.p, dt_of(storage), 0, h->stream, f));
    HIPCHK(launch_pack(d, h->ldp, k, H_B, ldb, h->P.p, dt_of(storage), n, h->stream, f));
  }
  const void* Pm = h->P.p;
  if (storage != EDA_F64) {
    STCHK(ensure(h, h->P64, (size_t)h->ldp * N * 8));
    HIPCHK(launch_pack(d, h->ldp, n, H_W, ldw, h->P64.p, DT::F64, 0, h->stream, nf));
    HIPCHK(launch_pack(d, h->ldp, k, H_B, ldb, h->P64.p, DT::F64, n, h->stream, nf));
    Pm = h->P64.p;
  }
  HIPCHK(hipMemcpyAsync(pin, h->flags.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  if (storage == EDA_FP8_E4M3) {
    STCHK(ensure(h, h->pscale, (size_t)N * 8));
    HIPCHK(launch_pack_fp8(d, h->ldp, N, h->P64.d(), h->pscale.d(), h->P.p, h->stream));
  }

  // a2: Gram G = P^T P in float64 (from the float64 factors)
  const int64_t gc = gram_chunks(d, N);
  STCHK(ensure(h, h->part, (size_t)gc * N * N * 8));
  STCHK(ensure(h, h->G, (size_t)N * N * 8));
  HIPCHK(launch_gram_partial(d, N, Pm, DT::F64, h->ldp, h->part.d(), gc, h->stream));
  HIPCHK(launch_gram_reduce(N, gc, h->part.d(), h->G.d(), N, h->stream));

  // a3: eig(H_B^T H_B) (core of exp(S_B) and the shift).  The W-cores come
  // from a matrix polynomial (poly_core_W) unless EDA_WCORE=eig selects
  // eig(H_W^T H_W) + phi weights; both routes are exact up to rounding.
  const char* wc = std::getenv("EDA_WCORE");
  const bool w_by_eig = (wc != nullptr && std::strcmp(wc, "eig") == 0);
  h->prep_wbyeig = w_by_eig;
  STCHK(ensure(h, h->eigW, (size_t)2 * n * 8));
  STCHK(ensure(h, h->eigZ, (size_t)2 * n * n * 8));
  STCHK(ensure(h, h->normbuf, 64));
  h->w_eig = false;
  h->prep_overlap = overlap && !w_by_eig;
  if (w_by_eig) {
    int hns[2] = {(int)n, (int)k};
    STCHK(ensure(h, h->nsbuf, 2 * sizeof(int)));
    HIPCHK(hipMemcpy(h->nsbuf.p, hns, sizeof(hns), hipMemcpyHostToDevice));
    STCHK(ensure(h, h->syev_work, 2 * syev_work_bytes(n)));
    HIPCHK(launch_syev(2, n, h->nsbuf.i(), h->G.d(), N, n + n * N, h->eigW.d(), n, h->eigZ.d(),
                       n, n * n, 0, h->syev_work.d(), h->stream));
    HIPCHK(hipMemcpyAsync(pin + 2 + k, h->eigW.d(), n * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(launch_norm1(n, h->G.d(), N, h->normbuf.d(), h->stream));
    HIPCHK(hipMemcpyAsync(pin + 2, h->eigW.d() + n, k * 8, hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipMemcpyAsync(pin + 1, h->normbuf.d(), 8, hipMemcpyDeviceToHost, h->stream));
    return EDA_OK;
  }
  // ||H_W^T H_W||_1 first: the W-cores need nothing else
  HIPCHK(launch_norm1(n, h->G.d(), N, h->normbuf.d(), h->stream));
  HIPCHK(hipMemcpyAsync(pin + 1, h->normbuf.d(), 8, hipMemcpyDeviceToHost, h->stream));
  hipStream_t sb = h->stream;
  if (h->prep_overlap) {
    if (h->aux == nullptr) HIPCHK(hipStreamCreateWithFlags(&h->aux, hipStreamNonBlocking));
    HIPCHK(hipEventRecord(h->prep_ev[2], h->stream));
    HIPCHK(hipStreamWaitEvent(h->aux, h->prep_ev[2], 0));
    sb = h->aux;
  }
  STCHK(ensure(h, h->syev_work, syev_work_bytes(k)));
  HIPCHK(launch_syev(1, k, nullptr, h->G.d() + n + n * N, N, 0, h->eigW.d() + n, 0,
                     h->eigZ.d() + n * n, n, 0, 0, h->syev_work.d(), sb));
  HIPCHK(hipMemcpyAsync(pin + 2, h->eigW.d() + n, k * 8, hipMemcpyDeviceToHost, sb));
  if (h->prep_overlap) HIPCHK(hipEventRecord(h->prep_ev[3], sb));
  return EDA_OK;
}

double prepare_time_ms(eda_handle h) {
  if (h->prep_time_pending) {
    float ms = 0.f;
    if (hipEventSynchronize(h->prep_ev[1]) == hipSuccess &&
        hipEventElapsedTime(&ms, h->prep_ev[0], h->prep_ev[1]) == hipSuccess)
      h->t_prepare_ms = ms;
    h->prep_time_pending = false;
  }
  return h->t_prepare_ms;
}

eda_status prepare_end(eda_handle h) {
  const double* pin = (const double*)h->pin;
  const int64_t n = h->n, k = h->k;
  int bad = 0;
  std::memcpy(&bad, pin, sizeof(int));
  if (bad) {
    if (h->prep_overlap) (void)hipEventSynchronize(h->prep_ev[3]);
    return fail(h, EDA_ERR_NONFINITE, "NaN or Inf in H_W or H_B");
  }
  h->normW = pin[1];
  if (h->prep_overlap) {
    // the W-cores while eig(H_B^T H_B) runs on the second stream
    STCHK(build_w_cores(h));
    HIPCHK(hipEventSynchronize(h->prep_ev[3]));
    HIPCHK(hipStreamWaitEvent(h->stream, h->prep_ev[3], 0));
  }
  h->hwB.assign(pin + 2, pin + 2 + k);
  if (h->prep_wbyeig) {
    h->hwW.assign(pin + 2 + k, pin + 2 + k + n);
    h->w_eig = true;
  }
  double lbmax = 0.0;
  for (double v : h->hwB) lbmax = std::max(lbmax, v);
  h->shiftB = lbmax;  // s = lambda_max(S_B): every factor e^{lambda - s} <= 1
  h->alphaB = std::exp(-h->shiftB);
  STCHK(ensure(h, h->alphaB_dev, 8));
  HIPCHK(launch_fill(1, h->alphaB, h->alphaB_dev.d(), h->stream));
  if (!h->prep_overlap) STCHK(build_w_cores(h));
  STCHK(build_composite_cores(h));
  HIPCHK(hipEventRecord(h->prep_ev[1], h->stream));
  h->prepared = true;
  return EDA_OK;
}

}  // namespace eda

extern "C" {

eda_status eda_prepare(eda_handle h, int64_t d, int64_t n, int64_t k, const double* H_W,
                       int64_t ldw, const double* H_B, int64_t ldb, eda_dtype storage) {
  if (h == nullptr) return EDA_ERR_ARG;
  STCHK(prepare_begin(h, d, n, k, H_W, ldw, H_B, ldb, storage, true));
  // the factors have been copied and checked once this returns: H_W and
  // H_B are not read after it
  HIPCHK(hipStreamSynchronize(h->stream));
  STCHK(prepare_end(h));
  // the cores are still being built on the stream; later calls on the
  // handle are ordered after them, so the host does not wait here
  h->prep_time_pending = true;
  return EDA_OK;
}

eda_status eda_expmv(eda_handle h, eda_which which, double c, int64_t b, const void* V,
                     int64_t ldv, void* Out, int64_t ldo, eda_dtype vdtype, double* log_scale) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (which != EDA_W && which != EDA_B) return fail(h, EDA_ERR_ARG, "which must be EDA_W or EDA_B");
  if (!std::isfinite(c)) return fail(h, EDA_ERR_ARG, "c must be finite");
  if (!h->prepared) return fail(h, EDA_ERR_STATE, "eda_prepare has not succeeded");
  STCHK(validate_block(h, b, V, ldv, Out, ldo, vdtype));
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, V, "V"));
  STCHK(check_dev_ptr(h, Out, "Out"));
  if (which == EDA_W && c > 0.0) STCHK(ensure_w_eig(h));  // the shift needs lambda_max
  const std::vector<double>& lam = which == EDA_W ? h->hwW : h->hwB;
  double lmax = 0.0;
  for (double v : lam) lmax = std::max(lmax, v);
  const double shift = c > 0.0 ? c * lmax : 0.0;
  const int64_t Nw = which == EDA_W ? h->n : h->k;
  CoreEntry* ce = nullptr;
  for (auto& e : h->cores)
    if (e.which == (int)which && e.c == c) ce = &e;
  if (ce == nullptr) {
    if (h->cores.size() >= 6) {
      HIPCHK(hipStreamSynchronize(h->stream));
      release(h->cores.front().buf);
      h->cores.erase(h->cores.begin());
    }
    h->cores.emplace_back();
    ce = &h->cores.back();
    ce->which = (int)which;
    ce->c = c;
    ce->shift = shift;
    STCHK(ensure(h, ce->buf, (size_t)Nw * Nw * 8));
    STCHK(build_core(h, (int)which, c, shift, ce->buf.d()));
  }
  const int64_t c0 = which == EDA_W ? 0 : h->n;
  STCHK(expop(h, false, c0, Nw, ce->buf.d(), Nw, std::exp(-shift), b, V, dt_of(vdtype), ldv, Out,
              dt_of(vdtype), ldo));
  if (log_scale != nullptr) *log_scale = shift;
  return EDA_OK;
}

eda_status eda_opmv(eda_handle h, eda_form form, int64_t b, const void* V, int64_t ldv,
                    void* Out, int64_t ldo, eda_dtype vdtype, double* log_scale) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (form != EDA_FORM_LANCZOS_M && form != EDA_FORM_ARNOLDI_A)
    return fail(h, EDA_ERR_ARG, "unknown operator form");
  if (!h->prepared) return fail(h, EDA_ERR_STATE, "eda_prepare has not succeeded");
  STCHK(validate_block(h, b, V, ldv, Out, ldo, vdtype));
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, V, "V"));
  STCHK(check_dev_ptr(h, Out, "Out"));
  if (form == EDA_FORM_ARNOLDI_A) STCHK(ensure_arnoldi_core(h));
  const double* C = form == EDA_FORM_LANCZOS_M ? h->CM.d() : h->CA.d();
  STCHK(expop(h, false, 0, h->N, C, h->N, h->alphaB, b, V, dt_of(vdtype), ldv, Out, dt_of(vdtype), ldo));
  if (log_scale != nullptr) *log_scale = h->shiftB;
  return EDA_OK;
}

eda_status eda_gram(eda_handle h, double* G, int64_t ldg) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (!h->prepared) return fail(h, EDA_ERR_STATE, "eda_prepare has not succeeded");
  if (G == nullptr || ldg < h->N) return fail(h, EDA_ERR_ARG, "G null or ldg < N");
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, G, "G"));
  HIPCHK(launch_copy_block(h->N, h->N, 1.0, h->G.d(), h->N, false, G, ldg, h->stream));
  return EDA_OK;
}

eda_status eda_factor_codes(eda_handle h, void* out, int64_t ldo, double* scales) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (!h->prepared) return fail(h, EDA_ERR_STATE, "eda_prepare has not succeeded");
  if (out == nullptr || ldo < h->d) return fail(h, EDA_ERR_ARG, "out null or ldo < d");
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, out, "out"));
  const size_t es = dsize(h->storage);
  HIPCHK(hipMemcpy2DAsync(out, (size_t)ldo * es, h->P.p, (size_t)h->ldp * es, (size_t)h->d * es,
                          (size_t)h->N, hipMemcpyDeviceToDevice, h->stream));
  if (scales != nullptr && h->storage == EDA_FP8_E4M3) {
    STCHK(check_dev_ptr(h, scales, "scales"));
    HIPCHK(hipMemcpyAsync(scales, h->pscale.p, (size_t)h->N * 8, hipMemcpyDeviceToDevice,
                          h->stream));
  }
  return EDA_OK;
}

eda_status eda_syev(eda_handle h, int64_t n, const double* A, int64_t lda, double* w, double* Z,
                    int64_t ldz) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (n < 1 || n > 2048) return fail(h, EDA_ERR_ARG, "n must be in [1, 2048]");
  if (A == nullptr || w == nullptr || Z == nullptr) return fail(h, EDA_ERR_ARG, "null pointer");
  if (lda < n || ldz < n) return fail(h, EDA_ERR_ARG, "lda/ldz must be >= n");
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, A, "A"));
  STCHK(check_dev_ptr(h, w, "w"));
  STCHK(check_dev_ptr(h, Z, "Z"));
  STCHK(ensure(h, h->syev_work, syev_work_bytes(n)));
  HIPCHK(launch_syev(1, n, nullptr, A, lda, 0, w, 0, Z, ldz, 0, 0, h->syev_work.d(), h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  return EDA_OK;
}

}  // extern "C"
