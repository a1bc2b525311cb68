// libeda host library: handle, validation, preprocessing, exponential
// products and the block Lanczos driver.  Every numerical step runs in the
// kernels of this directory; the host only validates, allocates, orders
// launches on the handle's stream and takes the small scalar decisions
// (spectral shift, convergence, restart).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "common.h"
#include "eda.h"

using namespace eda;

namespace {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
  double* d() const { return (double*)p; }
  int* i() const { return (int*)p; }
};

struct CoreEntry {
  int which = -1;
  double c = 0.0;
  double shift = 0.0;
  Buf buf;
};

}  // namespace

struct eda_handle_s {
  // events bracketing the operator products of a solve (reused across solves)
  std::vector<hipEvent_t> op_ev;
  size_t op_used = 0;
  hipStream_t stream = nullptr;
  int device = -1;
  std::string err;

  // prepared problem
  bool prepared = false;
  int64_t d = 0, n = 0, k = 0, N = 0, ldp = 0;
  eda_dtype storage = EDA_F64;
  Buf P, G, eigW, eigZ, nsbuf, Gh, Gm, GBs, CM, CA, T1, T2, T3, T4, fw, polyws, normbuf;
  double shiftB = 0.0, alphaB = 1.0;
  double normW = 0.0;   // ||H_W^T H_W||_1
  bool w_eig = false;   // eigenpairs of H_W^T H_W available
  std::vector<double> hwW, hwB;
  double t_prepare_ms = 0.0;

  // workspaces
  Buf part, Ysm, Zsm, syev_work, offs, flags, mask;
  std::vector<CoreEntry> cores;

  // solver
  Buf Q[2], H[2], Wb, T, wT, S, Sd, hz, Gs, Rinv, R1, Yb, MYb, dtheta, dres;
};

namespace {

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53

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

#define HIPCHK(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess)                                                           \
      return fail(h, EDA_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_));      \
  } while (0)

#define STCHK(x)                 \
  do {                           \
    eda_status s_ = (x);         \
    if (s_ != EDA_OK) return s_; \
  } while (0)

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

size_t dsize(eda_dtype t) { return t == EDA_F64 ? 8 : 4; }
DT dt_of(eda_dtype t) { return t == EDA_F64 ? DT::F64 : DT::F32; }

int64_t round_up(int64_t x, int64_t m) { return ((x + m - 1) / m) * m; }

// Low-rank exponential apply on columns [c0, c0+Nc) of P:
//   Out = alpha V + P_c (C (P_c^T V)),  C: Nc x Nc (ldc).
eda_status expop(eda_handle h, int64_t c0, int64_t Nc, const double* C, int64_t ldc,
                 double alpha, int64_t b, const void* V, DT vdt, int64_t ldv, void* Out,
                 DT odt, int64_t ldo) {
  const DT pdt = dt_of(h->storage);
  const char* Pc = (const char*)h->P.p + (size_t)c0 * h->ldp * dsize(h->storage);
  const int64_t chunks = tn_chunks(h->d, Nc, b);
  STCHK(ensure(h, h->part, (size_t)chunks * Nc * b * 8));
  STCHK(ensure(h, h->Ysm, (size_t)Nc * b * 8));
  STCHK(ensure(h, h->Zsm, (size_t)Nc * b * 8));
  HIPCHK(launch_tn_partial(h->d, Nc, b, Pc, pdt, h->ldp, V, vdt, ldv, h->part.d(), chunks,
                           nullptr, h->stream));
  // Y = P_c^T V (row-major, leading dimension b), then Z = C Y (row-major) by
  // the same streaming kernel with C as the tall operand
  HIPCHK(launch_reduce_partials(chunks, Nc, b, h->part.d(), 0.0, 0.0, nullptr, 0, 1.0,
                                h->Ysm.d(), b, nullptr, h->stream));
  HIPCHK(launch_nn(Nc, Nc, b, C, DT::F64, ldc, h->Ysm.d(), b, 0.0, nullptr, DT::F64, 0,
                   h->Zsm.d(), DT::F64, b, nullptr, h->stream, true));
  HIPCHK(launch_nn(h->d, Nc, b, Pc, pdt, h->ldp, h->Zsm.d(), b, alpha, V, vdt, ldv, Out, odt,
                   ldo, nullptr, h->stream));
  return EDA_OK;
}

// Core V diag(f) V^T of exp(c H H^T) e^{-shift} for the factor `which`.
// W-core by a matrix polynomial instead of an eigendecomposition:
//   G_c = c psi(c G_WW),  psi(X) = sum_{j>=0} X^j / (j+1)!  (psi(z) = (e^z - 1)/z),
// which equals V diag(phi_c(lambda)) V^T.  X = c G_WW / 2^q with ||X||_1 <= 1,
// psi(X) by Paterson-Stockmeyer (degree 17, truncation below 1/19! < 1e-17),
// then q doublings psi(2X) = psi(X) + psi(X) X psi(X) / 2.  Only GEMMs.
eda_status poly_core_W(eda_handle h, double c, double* out) {
  const int64_t n = h->n, N = h->N, nn = n * n;
  hipStream_t s = h->stream;
  STCHK(ensure(h, h->polyws, (size_t)7 * nn * 8));
  double* X = h->polyws.d();
  double* A2 = X + nn;
  double* A3 = A2 + nn;
  double* A4 = A3 + nn;
  double* P = A4 + nn;
  double* T = P + nn;
  double* U = T + nn;
  double nrm = std::fabs(c) * h->normW;
  int q = 0;
  while (nrm > 1.0 && q < 60) {
    nrm *= 0.5;
    ++q;
  }
  const double sc = c * std::ldexp(1.0, -q);
  double a[18];
  double f = 1.0;
  for (int j = 0; j < 18; ++j) {
    f *= (double)(j + 1);
    a[j] = 1.0 / f;  // 1/(j+1)!
  }
  HIPCHK(launch_copy_block(n, n, sc, h->G.d(), N, false, X, n, s));
  HIPCHK(launch_gemm(false, false, n, n, n, 1.0, X, n, nullptr, X, n, 0.0, A2, n, s));
  HIPCHK(launch_gemm(false, false, n, n, n, 1.0, A2, n, nullptr, X, n, 0.0, A3, n, s));
  HIPCHK(launch_gemm(false, false, n, n, n, 1.0, A2, n, nullptr, A2, n, 0.0, A4, n, s));
  HIPCHK(launch_lincomb(n, a[16], a[17], X, 0.0, nullptr, 0.0, nullptr, n, P, n, s));
  for (int kb = 3; kb >= 0; --kb) {
    HIPCHK(launch_lincomb(n, a[4 * kb], a[4 * kb + 1], X, a[4 * kb + 2], A2, a[4 * kb + 3], A3,
                          n, T, n, s));
    HIPCHK(launch_gemm(false, false, n, n, n, 1.0, A4, n, nullptr, P, n, 1.0, T, n, s));
    std::swap(P, T);
  }
  for (int i = 0; i < q; ++i) {
    HIPCHK(launch_gemm(false, false, n, n, n, 1.0, X, n, nullptr, P, n, 0.0, U, n, s));
    HIPCHK(launch_copy_block(n, n, 1.0, P, n, false, T, n, s));
    HIPCHK(launch_gemm(false, false, n, n, n, 0.5, P, n, nullptr, U, n, 1.0, T, n, s));
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
  HIPCHK(launch_gemm(false, true, Nw, Nw, Nw, 1.0, Z, ldz, h->fw.d(), Z, ldz, 0.0, out, Nw,
                     h->stream));
  return EDA_OK;
}

eda_status build_composite_cores(eda_handle h) {
  const int64_t n = h->n, k = h->k, N = h->N;
  STCHK(ensure(h, h->Gh, (size_t)n * n * 8));
  STCHK(ensure(h, h->Gm, (size_t)n * n * 8));
  STCHK(ensure(h, h->GBs, (size_t)k * k * 8));
  STCHK(ensure(h, h->CM, (size_t)N * N * 8));
  STCHK(ensure(h, h->CA, (size_t)N * N * 8));
  STCHK(ensure(h, h->T1, (size_t)n * k * 8));
  STCHK(ensure(h, h->T2, (size_t)n * k * 8));
  STCHK(ensure(h, h->T3, (size_t)n * k * 8));
  STCHK(ensure(h, h->T4, (size_t)n * k * 8));
  STCHK(build_core(h, EDA_W, -0.5, 0.0, h->Gh.d()));
  if (h->w_eig) {
    STCHK(build_core(h, EDA_W, -1.0, 0.0, h->Gm.d()));
  } else {
    // exp(-S_W) = exp(-S_W/2)^2 gives G_m = 2 G_h + G_h (H_W^T H_W) G_h
    HIPCHK(launch_gemm(false, false, n, n, n, 1.0, h->G.d(), N, nullptr, h->Gh.d(), n, 0.0,
                       h->CM.d(), n, h->stream));
    HIPCHK(launch_copy_block(n, n, 2.0, h->Gh.d(), n, false, h->Gm.d(), n, h->stream));
    HIPCHK(launch_gemm(false, false, n, n, n, 1.0, h->Gh.d(), n, nullptr, h->CM.d(), n, 1.0,
                       h->Gm.d(), n, h->stream));
  }
  STCHK(build_core(h, EDA_B, 1.0, h->shiftB, h->GBs.d()));
  const double* K = h->G.d() + n * N;  // H_W^T H_B, n x k, ld N
  hipStream_t s = h->stream;
  double* CM = h->CM.d();
  double* CA = h->CA.d();
  // Lanczos core: [[a Gm + Gh K GB K^T Gh, Gh K GB], [GB K^T Gh, GB]]
  HIPCHK(launch_gemm(false, false, n, k, n, 1.0, h->Gh.d(), n, nullptr, K, N, 0.0, h->T1.d(), n, s));
  HIPCHK(launch_gemm(false, false, n, k, k, 1.0, h->T1.d(), n, nullptr, h->GBs.d(), k, 0.0,
                     h->T2.d(), n, s));
  HIPCHK(launch_copy_block(n, n, h->alphaB, h->Gm.d(), n, false, CM, N, s));
  HIPCHK(launch_gemm(false, true, n, n, k, 1.0, h->T2.d(), n, nullptr, h->T1.d(), n, 1.0, CM, N, s));
  HIPCHK(launch_copy_block(n, k, 1.0, h->T2.d(), n, false, CM + n * N, N, s));
  HIPCHK(launch_copy_block(k, n, 1.0, h->T2.d(), n, true, CM + n, N, s));
  HIPCHK(launch_copy_block(k, k, 1.0, h->GBs.d(), k, false, CM + n + n * N, N, s));
  // Arnoldi core: [[a Gm, Gm K GB], [0, GB]]
  HIPCHK(launch_gemm(false, false, n, k, n, 1.0, h->Gm.d(), n, nullptr, K, N, 0.0, h->T3.d(), n, s));
  HIPCHK(launch_gemm(false, false, n, k, k, 1.0, h->T3.d(), n, nullptr, h->GBs.d(), k, 0.0,
                     h->T4.d(), n, s));
  HIPCHK(launch_copy_block(n, n, h->alphaB, h->Gm.d(), n, false, CA, N, s));
  HIPCHK(launch_copy_block(n, k, 1.0, h->T4.d(), n, false, CA + n * N, N, s));
  HIPCHK(launch_copy_block(k, n, 0.0, h->T4.d(), n, true, CA + n, N, s));
  HIPCHK(launch_copy_block(k, k, 1.0, h->GBs.d(), k, false, CA + n + n * N, N, s));
  return EDA_OK;
}

eda_status validate_block(eda_handle h, int64_t b, const void* V, int64_t ldv, const void* Out,
                          int64_t ldo, eda_dtype vdtype) {
  if (b < 1 || b > (1 << 20)) return fail(h, EDA_ERR_ARG, "block width b=%lld out of range", (long long)b);
  if (V == nullptr || Out == nullptr) return fail(h, EDA_ERR_ARG, "null V or Out");
  if (vdtype != EDA_F64 && vdtype != EDA_F32)
    return fail(h, EDA_ERR_ARG, "vdtype must be EDA_F64 or EDA_F32");
  if (h->storage == EDA_F64 && vdtype != EDA_F64)
    return fail(h, EDA_ERR_ARG, "float64 storage takes float64 blocks");
  if (ldv < h->d || ldo < h->d) return fail(h, EDA_ERR_ARG, "ldv/ldo must be >= d");
  const size_t es = dsize(vdtype);
  const char* v0 = (const char*)V;
  const char* v1 = v0 + ((b - 1) * ldv + h->d) * es;
  const char* o0 = (const char*)Out;
  const char* o1 = o0 + ((b - 1) * ldo + h->d) * es;
  if (v0 < o1 && o0 < v1) return fail(h, EDA_ERR_ARG, "V and Out overlap");
  return EDA_OK;
}

}  // namespace

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
                  &h->CM, &h->CA, &h->T1,   &h->T2,   &h->T3,    &h->T4,  &h->fw,  &h->part,
                  &h->Ysm, &h->Zsm, &h->syev_work, &h->offs, &h->flags, &h->mask, &h->Q[0], &h->Q[1],
                  &h->H[0], &h->H[1], &h->Wb, &h->T, &h->wT, &h->S, &h->Sd, &h->hz, &h->Gs,
                  &h->Rinv, &h->R1, &h->Yb, &h->MYb, &h->dtheta, &h->dres};
    for (Buf* b : all) release(*b);
    for (auto& c : h->cores) release(c.buf);
    for (hipEvent_t e : h->op_ev) (void)hipEventDestroy(e);
  }
  delete h;
}

eda_status eda_scatter_factors(eda_handle h, int64_t d, int64_t n, int64_t k, const double* X,
                               int64_t ldx, const int64_t* counts, double* H_W, int64_t ldw,
                               double* H_B, int64_t ldb) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (d < 1 || n < 1 || k < 1 || k > n) return fail(h, EDA_ERR_ARG, "need d>=1, 1<=k<=n");
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

eda_status eda_prepare(eda_handle h, int64_t d, int64_t n, int64_t k, const double* H_W,
                       int64_t ldw, const double* H_B, int64_t ldb, eda_dtype storage) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (d < 2 || k < 2 || n < k) return fail(h, EDA_ERR_ARG, "need d>=2, k>=2, n>=k");
  if (n + k > 2048) return fail(h, EDA_ERR_ARG, "n+k=%lld exceeds 2048", (long long)(n + k));
  if (H_W == nullptr || H_B == nullptr) return fail(h, EDA_ERR_ARG, "null factor");
  if (ldw < d || ldb < d) return fail(h, EDA_ERR_ARG, "leading dimensions must be >= d");
  if (storage != EDA_F64 && storage != EDA_F32)
    return fail(h, EDA_ERR_ARG, "storage must be EDA_F64 or EDA_F32");
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, H_W, "H_W"));
  STCHK(check_dev_ptr(h, H_B, "H_B"));
  h->prepared = false;
  for (auto& c : h->cores) release(c.buf);
  h->cores.clear();

  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, h->stream));

  const int64_t N = n + k;
  h->d = d;
  h->n = n;
  h->k = k;
  h->N = N;
  h->storage = storage;
  h->ldp = round_up(d, 64);

  STCHK(ensure(h, h->flags, 64));
  HIPCHK(launch_fill_i32(16, 0, h->flags.i(), h->stream));
  HIPCHK(launch_nonfinite(d, n, H_W, ldw, h->flags.i(), h->stream));
  HIPCHK(launch_nonfinite(d, k, H_B, ldb, h->flags.i(), h->stream));
  int bad = 0;
  HIPCHK(hipMemcpyAsync(&bad, h->flags.p, sizeof(int), hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (bad) {
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return fail(h, EDA_ERR_NONFINITE, "NaN or Inf in H_W or H_B");
  }

  // a1: factor ingest, P = [H_W H_B] in storage precision
  STCHK(ensure(h, h->P, (size_t)h->ldp * N * dsize(storage)));
  HIPCHK(launch_pack(d, h->ldp, n, H_W, ldw, h->P.p, dt_of(storage), 0, h->stream));
  HIPCHK(launch_pack(d, h->ldp, k, H_B, ldb, h->P.p, dt_of(storage), n, h->stream));

  // a2: Gram G = P^T P in float64
  const int64_t gc = gram_chunks(d, N);
  STCHK(ensure(h, h->part, (size_t)gc * N * N * 8));
  STCHK(ensure(h, h->G, (size_t)N * N * 8));
  HIPCHK(launch_gram_partial(d, N, h->P.p, dt_of(storage), h->ldp, h->part.d(), gc, h->stream));
  HIPCHK(launch_gram_reduce(N, gc, h->part.d(), h->G.d(), N, h->stream));

  // a3: eig(H_B^T H_B) (core of exp(S_B) and the shift).  The W-cores come
  // from a matrix polynomial (poly_core_W) unless EDA_WCORE=eig selects
  // eig(H_W^T H_W) + phi weights; both routes are exact up to rounding.
  const char* wc = std::getenv("EDA_WCORE");
  const bool w_by_eig = (wc != nullptr && std::strcmp(wc, "eig") == 0);
  STCHK(ensure(h, h->eigW, (size_t)2 * n * 8));
  STCHK(ensure(h, h->eigZ, (size_t)2 * n * n * 8));
  STCHK(ensure(h, h->normbuf, 64));
  h->w_eig = false;
  if (w_by_eig) {
    int hns[2] = {(int)n, (int)k};
    STCHK(ensure(h, h->nsbuf, 2 * sizeof(int)));
    HIPCHK(hipMemcpy(h->nsbuf.p, hns, sizeof(hns), hipMemcpyHostToDevice));
    STCHK(ensure(h, h->syev_work, 2 * syev_work_bytes(n)));
    HIPCHK(launch_syev(2, n, h->nsbuf.i(), h->G.d(), N, n + n * N, h->eigW.d(), n, h->eigZ.d(),
                       n, n * n, 0, h->syev_work.d(), h->stream));
    h->hwW.assign(n, 0.0);
    HIPCHK(hipMemcpyAsync(h->hwW.data(), h->eigW.d(), n * 8, hipMemcpyDeviceToHost, h->stream));
    h->w_eig = true;
  } else {
    STCHK(ensure(h, h->syev_work, syev_work_bytes(k)));
    HIPCHK(launch_syev(1, k, nullptr, h->G.d() + n + n * N, N, 0, h->eigW.d() + n, 0,
                       h->eigZ.d() + n * n, n, 0, 0, h->syev_work.d(), h->stream));
  }
  HIPCHK(launch_norm1(n, h->G.d(), N, h->normbuf.d(), h->stream));
  h->hwB.assign(k, 0.0);
  HIPCHK(hipMemcpyAsync(h->hwB.data(), h->eigW.d() + n, k * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(&h->normW, h->normbuf.d(), 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  double lbmax = 0.0;
  for (double v : h->hwB) lbmax = std::max(lbmax, v);
  h->shiftB = lbmax;  // s = lambda_max(S_B): every factor e^{lambda - s} <= 1
  h->alphaB = std::exp(-h->shiftB);

  STCHK(build_composite_cores(h));
  HIPCHK(hipEventRecord(e1, h->stream));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  h->t_prepare_ms = ms;
  h->prepared = true;
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
  STCHK(expop(h, c0, Nw, ce->buf.d(), Nw, std::exp(-shift), b, V, dt_of(vdtype), ldv, Out,
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
  const double* C = form == EDA_FORM_LANCZOS_M ? h->CM.d() : h->CA.d();
  STCHK(expop(h, 0, h->N, C, h->N, h->alphaB, b, V, dt_of(vdtype), ldv, Out, dt_of(vdtype), ldo));
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

// ---------------------------------------------------------------------------
// Block Lanczos (Algorithm 3 on the symmetric form M, eqs. (3.13)-(3.16))
// ---------------------------------------------------------------------------
namespace {

struct Solver {
  eda_handle h;
  int64_t d, ldq, b, mmax, ldh, t, kk;
  int cur = 0;  // which of the two basis/H buffers is live
  double* Q() const { return h->Q[cur].d(); }
  double* H() const { return h->H[cur].d(); }
};

// One Cholesky QR pass: G = X^T X, X_out = X R^{-1}.  Optionally records R
// (combined with Rprev) and raises the repair flag.
eda_status cholqr_pass(eda_handle h, int64_t d, int64_t cols, const double* X, int64_t ldx,
                       double* Xout, int64_t ldxo, const double* Rprev, double* Rout,
                       int64_t ldro, const double* hcol, int64_t mrows, int64_t ldhc,
                       const int* gate, int* flag) {
  const int64_t chunks = tn_chunks(d, cols, cols);
  STCHK(ensure(h, h->part, (size_t)chunks * cols * cols * 8));
  STCHK(ensure(h, h->Gs, (size_t)cols * cols * 8));
  STCHK(ensure(h, h->Rinv, (size_t)cols * cols * 8));
  HIPCHK(launch_tn_partial(d, cols, cols, X, DT::F64, ldx, X, DT::F64, ldx, h->part.d(), chunks,
                           gate, h->stream));
  HIPCHK(launch_reduce_partials(chunks, cols, cols, h->part.d(), 1.0, 0.0, h->Gs.d(), cols, 0.0,
                                nullptr, 0, gate, h->stream));
  HIPCHK(launch_chol(cols, h->Gs.d(), cols, h->Rinv.d(), cols, Rprev, cols, Rout, ldro, hcol,
                     mrows, ldhc, 1e-4, flag, gate, h->stream));
  HIPCHK(launch_nn(d, cols, cols, X, DT::F64, ldx, h->Rinv.d(), cols, 0.0, nullptr, DT::F64, ldx,
                   Xout, DT::F64, ldxo, gate, h->stream));
  return EDA_OK;
}

// One classical Gram-Schmidt pass of W against Q[:, 0:m]:
//   h = Q^T W (accumulated into Hcol when given),  W -= Q h.
eda_status cgs_pass(eda_handle h, int64_t d, int64_t m, const double* Q, int64_t ldq, double* W,
                    int64_t ldw, int64_t b, double* Hcol, int64_t ldh, double beta,
                    const int* gate) {
  const int64_t chunks = tn_chunks(d, m, b);
  STCHK(ensure(h, h->part, (size_t)chunks * m * b * 8));
  STCHK(ensure(h, h->hz, (size_t)m * b * 8));
  HIPCHK(launch_tn_partial(d, m, b, Q, DT::F64, ldq, W, DT::F64, ldw, h->part.d(), chunks, gate,
                           h->stream));
  HIPCHK(launch_reduce_partials(chunks, m, b, h->part.d(), 1.0, beta, Hcol, ldh, -1.0, h->hz.d(),
                                b, gate, h->stream));
  HIPCHK(launch_nn(d, m, b, Q, DT::F64, ldq, h->hz.d(), b, 1.0, W, DT::F64, ldw, W, DT::F64, ldw,
                   gate, h->stream));
  return EDA_OK;
}

// Block step: from the basis Q[:, 0:m+b] (current block Q[:, m:m+b]) build
// Q[:, m+b:m+2b] and column block m of H.
eda_status lanczos_step(Solver& S, int64_t m) {
  eda_handle h = S.h;
  const int64_t d = S.d, b = S.b, ldq = S.ldq, ldh = S.ldh;
  double* Q = S.Q();
  double* H = S.H();
  double* W = h->Wb.d();
  int* flags = h->flags.i();
  // W = e^{-s} M V_j, timed with a pair of events
  if (h->op_used + 2 > h->op_ev.size()) {
    for (int q = 0; q < 64; ++q) {
      hipEvent_t e;
      HIPCHK(hipEventCreate(&e));
      h->op_ev.push_back(e);
    }
  }
  HIPCHK(hipEventRecord(h->op_ev[h->op_used], h->stream));
  STCHK(expop(h, 0, h->N, h->CM.d(), h->N, h->alphaB, b, Q + m * ldq, DT::F64, ldq, W, DT::F64,
              ldq));
  HIPCHK(hipEventRecord(h->op_ev[h->op_used + 1], h->stream));
  h->op_used += 2;
  // CGS2 against Q[:, 0:m+b]
  double* Hcol = H + m * ldh;
  STCHK(cgs_pass(h, d, m + b, Q, ldq, W, ldq, b, Hcol, ldh, 0.0, nullptr));
  STCHK(cgs_pass(h, d, m + b, Q, ldq, W, ldq, b, Hcol, ldh, 1.0, nullptr));
  // Block orthonormalisation, R = R2 R1 going to H[m+b:m+2b, m:m+b].
  // Pass 1 is rank revealing: directions along which the Krylov space has
  // become invariant are deflated and replaced by fresh random directions
  // with zero coupling (their rows of R1 are zero).
  double* Qn = Q + (m + b) * ldq;
  {
    const int64_t chunks = tn_chunks(d, b, b);
    HIPCHK(launch_tn_partial(d, b, b, W, DT::F64, ldq, W, DT::F64, ldq, h->part.d(), chunks,
                             nullptr, h->stream));
    HIPCHK(launch_reduce_partials(chunks, b, b, h->part.d(), 1.0, 0.0, h->Gs.d(), b, 0.0, nullptr,
                                  0, nullptr, h->stream));
    HIPCHK(launch_pchol(b, h->Gs.d(), b, Hcol, m + b, ldh, 1e-13, 1e-4, h->Rinv.d(), b,
                        h->R1.d(), b, h->mask.i(), flags, h->stream));
    HIPCHK(launch_nn(d, b, b, W, DT::F64, ldq, h->Rinv.d(), b, 0.0, nullptr, DT::F64, ldq, Qn,
                     DT::F64, ldq, nullptr, h->stream));
    HIPCHK(launch_fill_masked_randn(d, b, h->mask.i(), 0x5eed0000ull + (uint64_t)m, Qn, ldq,
                                    h->stream));
  }
  STCHK(cholqr_pass(h, d, b, Qn, ldq, Qn, ldq, h->R1.d(), H + (m + b) + m * ldh, ldh, nullptr, 0,
                    0, nullptr, flags));
  // repair (only runs when the flag was raised): re-orthogonalise the new block
  STCHK(cgs_pass(h, d, m + b, Q, ldq, Qn, ldq, b, nullptr, 0, 0.0, flags));
  STCHK(cgs_pass(h, d, m + b, Q, ldq, Qn, ldq, b, nullptr, 0, 0.0, flags));
  STCHK(cholqr_pass(h, d, b, Qn, ldq, Qn, ldq, nullptr, nullptr, 0, nullptr, 0, 0, flags, nullptr));
  STCHK(cholqr_pass(h, d, b, Qn, ldq, Qn, ldq, nullptr, nullptr, 0, nullptr, 0, 0, flags, nullptr));
  HIPCHK(launch_flag_fold(flags, h->stream));
  return EDA_OK;
}

// Rayleigh-Ritz on Q[:, 0:m]: eigenpairs of sym(H[0:m,0:m]); returns the top
// `cnt` Ritz values (descending) and residual estimates on the host.
eda_status rayleigh_ritz(Solver& S, int64_t m, int64_t nvec, int64_t cnt, double* theta,
                         double* est) {
  eda_handle h = S.h;
  const int64_t ldh = S.ldh, mm = S.mmax;
  HIPCHK(launch_symmetrize(m, S.H(), ldh, h->T.d(), mm, h->stream));
  HIPCHK(launch_syev(1, m, nullptr, h->T.d(), mm, 0, h->wT.d(), 0, h->S.d(), mm, 0, nvec,
                     h->syev_work.d(), h->stream));
  const double* Bm = S.H() + m + (m - S.b) * ldh;
  HIPCHK(launch_ritz_estimates(m, S.b, cnt, h->wT.d(), h->S.d(), mm, Bm, ldh, h->dtheta.d(),
                               h->dres.d(), h->stream));
  HIPCHK(hipMemcpyAsync(theta, h->dtheta.d(), cnt * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipMemcpyAsync(est, h->dres.d(), cnt * 8, hipMemcpyDeviceToHost, h->stream));
  HIPCHK(hipStreamSynchronize(h->stream));
  if (std::getenv("EDA_LOG") != nullptr) {
    int fl[2] = {0, 0};
    HIPCHK(hipMemcpy(fl, h->flags.p, sizeof(fl), hipMemcpyDeviceToHost));
    std::fprintf(stderr, "[eda] rr m=%lld cnt=%lld flags=%d/%d theta:", (long long)m,
                 (long long)cnt, fl[0], fl[1]);
    for (int64_t i = 0; i < cnt; ++i) std::fprintf(stderr, " %.6e", theta[i]);
    std::fprintf(stderr, "\n[eda]   est:");
    for (int64_t i = 0; i < cnt; ++i) std::fprintf(stderr, " %.2e", est[i]);
    std::fprintf(stderr, "\n");
  }
  return EDA_OK;
}

}  // namespace

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
  if (o.form != EDA_FORM_LANCZOS_M) return fail(h, EDA_ERR_ARG, "only the Lanczos form is solved");
  if (o.krylov_dtype != EDA_F64 || o.refine_dtype != EDA_F64)
    return fail(h, EDA_ERR_ARG, "Krylov and refinement arithmetic must be EDA_F64");
  if (o.resmode != EDA_RES_REL_THETA && o.resmode != EDA_RES_NORMWISE)
    return fail(h, EDA_ERR_ARG, "unknown residual mode");
  const int64_t b = o.block > 0 ? o.block : 8;
  if (b > 8) return fail(h, EDA_ERR_ARG, "block width must be in [1, 8]");
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
  const int64_t check_every = o.check_every > 0 ? o.check_every : 2;
  if (o.start_block != nullptr && o.ld_start < d)
    return fail(h, EDA_ERR_ARG, "ld_start must be >= d");
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, X, "X"));
  if (o.start_block != nullptr) STCHK(check_dev_ptr(h, o.start_block, "start_block"));

  Solver S;
  S.h = h;
  S.d = d;
  S.ldq = h->ldp;
  S.b = b;
  S.mmax = mmax;
  S.ldh = mmax + b;
  S.t = t;
  S.kk = std::min<int64_t>(t + b, mmax - 2 * b);
  if (S.kk < t) S.kk = t;
  const int64_t ldq = S.ldq, ldh = S.ldh;

  for (int q = 0; q < 2; ++q) {
    STCHK(ensure(h, h->Q[q], (size_t)ldq * (mmax + b) * 8));
    STCHK(ensure(h, h->H[q], (size_t)ldh * ldh * 8));
  }
  STCHK(ensure(h, h->Wb, (size_t)ldq * std::max<int64_t>(b, t) * 8));
  STCHK(ensure(h, h->T, (size_t)mmax * mmax * 8));
  STCHK(ensure(h, h->wT, (size_t)mmax * 8));
  STCHK(ensure(h, h->S, (size_t)mmax * mmax * 8));
  STCHK(ensure(h, h->Sd, (size_t)mmax * S.kk * 8));
  STCHK(ensure(h, h->Yb, (size_t)ldq * t * 8));
  STCHK(ensure(h, h->MYb, (size_t)ldq * t * 8));
  STCHK(ensure(h, h->dtheta, (size_t)(S.kk + 8) * 8));
  STCHK(ensure(h, h->dres, (size_t)(S.kk + 8) * 8));
  STCHK(ensure(h, h->syev_work, syev_work_bytes(mmax)));
  STCHK(ensure(h, h->flags, 64));
  STCHK(ensure(h, h->mask, 64 * sizeof(int)));
  {
    // size the shared workspaces once for every shape used below
    const int64_t bt = std::max<int64_t>(b, t);
    const int64_t shapes[][2] = {{h->N, b}, {mmax + b, b}, {b, b}, {h->N, t}, {h->n, t}, {t, t}};
    size_t pmax = 0;
    for (const auto& sh : shapes)
      pmax = std::max(pmax, (size_t)tn_chunks(d, sh[0], sh[1]) * sh[0] * sh[1] * 8);
    STCHK(ensure(h, h->part, pmax));
    STCHK(ensure(h, h->Ysm, (size_t)h->N * bt * 8));
    STCHK(ensure(h, h->Zsm, (size_t)h->N * bt * 8));
    STCHK(ensure(h, h->hz, (size_t)(mmax + b) * b * 8));
    STCHK(ensure(h, h->Gs, (size_t)bt * bt * 8));
    STCHK(ensure(h, h->Rinv, (size_t)bt * bt * 8));
    STCHK(ensure(h, h->R1, (size_t)b * b * 8));
  }

  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  HIPCHK(hipEventRecord(e0, h->stream));
  hipStream_t s = h->stream;
  h->op_used = 0;
  HIPCHK(launch_fill_i32(16, 0, h->flags.i(), s));
  HIPCHK(launch_fill(ldh * ldh, 0.0, h->H[0].d(), s));
  HIPCHK(launch_fill(ldh * ldh, 0.0, h->H[1].d(), s));
  S.cur = 0;

  // start block -> Q[:, 0:b]
  double* Wst = h->Wb.d();
  if (o.start_block != nullptr)
    HIPCHK(launch_copy2d(d, b, o.start_block, DT::F64, o.ld_start, Wst, DT::F64, ldq, s));
  else
    HIPCHK(launch_randn(d, b, o.seed, Wst, ldq, s));
  HIPCHK(launch_fill(ldq * (mmax + b), 0.0, S.Q(), s));
  STCHK(cholqr_pass(h, d, b, Wst, ldq, S.Q(), ldq, nullptr, nullptr, 0, nullptr, 0, 0, nullptr,
                    nullptr));
  STCHK(cholqr_pass(h, d, b, S.Q(), ldq, S.Q(), ldq, nullptr, nullptr, 0, nullptr, 0, 0, nullptr,
                    nullptr));

  const int64_t nvec = std::min<int64_t>(S.kk, mmax);
  std::vector<double> theta(S.kk + 8), est(S.kk + 8);
  int64_t m = 0;
  int64_t iters = 0, restarts = 0;
  bool converged = false;
  int flags_out = 0;
  if (t > h->k - 1) flags_out |= EDA_WARN_DEGENERATE;
  double bytes = 0.0;
  int64_t ops = 0;
  const double opbytes = 2.0 * d * h->N * dsize(h->storage) + 3.0 * d * b * 8.0;
  bool floor_limited = false;
  int64_t m_rr = 0;

  while (true) {
    STCHK(lanczos_step(S, m));
    m += b;
    ++iters;
    ops += b;
    bytes += opbytes;
    const bool need_restart = (m + b > mmax);
    const bool can_check = (m >= t + b) || need_restart;
    if (can_check && (iters % check_every == 0 || need_restart || iters >= max_iter)) {
      const int64_t cnt = need_restart ? S.kk : t;
      STCHK(rayleigh_ritz(S, m, std::min<int64_t>(nvec, m), cnt, theta.data(), est.data()));
      m_rr = m;
      bool ok = true;
      floor_limited = false;
      const double th1 = theta[0];
      for (int64_t i = 0; i < t; ++i) {
        const double thi = theta[i];
        if (!(thi > 0.0)) { ok = false; continue; }
        const double floor_i = 10.0 * kU64 * th1 / thi;
        const double tol_i = std::max(tol, floor_i);
        if (floor_i > tol) floor_limited = true;
        const double r = (o.resmode == EDA_RES_REL_THETA) ? est[i] / thi : est[i] / th1;
        if (!(r <= tol_i)) ok = false;
      }
      if (ok) { converged = true; break; }
      if (iters >= max_iter) break;
      if (need_restart) {
        // thick restart: keep the kk leading Ritz vectors and the next block
        const int64_t kk = S.kk;
        HIPCHK(launch_gather_desc(m, kk, h->S.d(), mmax, h->Sd.d(), kk, s));
        const int nxt = 1 - S.cur;
        double* Qn = h->Q[nxt].d();
        double* Hn = h->H[nxt].d();
        HIPCHK(launch_nn(d, m, kk, S.Q(), DT::F64, ldq, h->Sd.d(), kk, 0.0, nullptr, DT::F64, ldq,
                         Qn, DT::F64, ldq, nullptr, s));
        HIPCHK(launch_copy2d(d, b, S.Q() + m * ldq, DT::F64, ldq, Qn + kk * ldq, DT::F64, ldq, s));
        HIPCHK(launch_fill(ldh * ldh, 0.0, Hn, s));
        HIPCHK(launch_set_diag(kk, h->dtheta.d(), Hn, ldh, s));
        HIPCHK(launch_restart_coupling(m, b, kk, S.H() + m + (m - b) * ldh, ldh, h->Sd.d(), kk, Hn,
                                       ldh, s));
        S.cur = nxt;
        m = kk;
        ++restarts;
      }
    } else if (iters >= max_iter) {
      STCHK(rayleigh_ritz(S, m, std::min<int64_t>(nvec, m), std::min<int64_t>(t, m), theta.data(),
                          est.data()));
      m_rr = m;
      break;
    }
  }
  if (m_rr != m || m < t) {
    // final Rayleigh-Ritz on the current basis
    if (m < t) return fail(h, EDA_ERR_NOCONV, "basis smaller than t at the iteration limit");
    STCHK(rayleigh_ritz(S, m, std::min<int64_t>(nvec, m), t, theta.data(), est.data()));
  }

  // Ritz vectors Y = Q S_t, explicit residuals, back-transform x = exp(-S_W/2) y
  HIPCHK(launch_gather_desc(m, t, h->S.d(), mmax, h->Sd.d(), t, s));
  double* Y = h->Yb.d();
  double* MY = h->MYb.d();
  HIPCHK(launch_nn(d, m, t, S.Q(), DT::F64, ldq, h->Sd.d(), t, 0.0, nullptr, DT::F64, ldq, Y,
                   DT::F64, ldq, nullptr, s));
  STCHK(expop(h, 0, h->N, h->CM.d(), h->N, h->alphaB, t, Y, DT::F64, ldq, MY, DT::F64, ldq));
  ops += t;
  bytes += 2.0 * d * h->N * dsize(h->storage) + 3.0 * d * t * 8.0;
  HIPCHK(launch_ritz_residual(d, t, MY, Y, ldq, DT::F64, h->dtheta.d(), h->dres.d(), s));
  HIPCHK(hipEventRecord(e1, s));
  STCHK(expop(h, 0, h->n, h->Gh.d(), h->n, 1.0, t, Y, DT::F64, ldq, X, DT::F64, ldx));
  // orthonormalise X in decreasing-lambda order (Cholesky QR, twice), then signs
  STCHK(cholqr_pass(h, d, t, X, ldx, MY, ldq, nullptr, nullptr, 0, nullptr, 0, 0, nullptr, nullptr));
  STCHK(cholqr_pass(h, d, t, MY, ldq, X, ldx, nullptr, nullptr, 0, nullptr, 0, 0, nullptr, nullptr));
  HIPCHK(launch_sign_fix(d, t, X, ldx, s));
  std::vector<double> res(t);
  int fl[2] = {0, 0};
  HIPCHK(hipMemcpyAsync(theta.data(), h->dtheta.d(), t * 8, hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(res.data(), h->dres.d(), t * 8, hipMemcpyDeviceToHost, s));
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
  if (floor_limited) flags_out |= EDA_WARN_FLOOR;
  if (fl[1] | fl[0]) flags_out |= EDA_WARN_REPAIRED;
  if (info != nullptr) {
    info->iters = (int32_t)iters;
    info->restarts = (int32_t)restarts;
    info->refine_passes = 0;
    info->flags = flags_out;
    info->ops = ops;
    info->bytes_moved = bytes;
    info->t_prepare_ms = h->t_prepare_ms;
    info->t_krylov_ms = kms;
    info->t_refine_ms = 0.0;
    info->shift_s = h->shiftB;
    double top = 0.0;
    for (size_t q = 0; q + 1 < h->op_used; q += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, h->op_ev[q], h->op_ev[q + 1]) == hipSuccess) top += ms;
    }
    info->op_calls = (int64_t)(h->op_used / 2);
    info->t_op_ms = top;
    info->op_bytes = 2.0 * d * h->N * dsize(h->storage) + 3.0 * d * b * 8.0;
  }
  if (range_err) return fail(h, EDA_ERR_RANGE, "a Ritz value underflowed after the shift");
  if (!converged) return fail(h, EDA_ERR_NOCONV, "max_iter reached before convergence");
  return EDA_OK;
}
