// eda_opmv_noalloc: the composite exponential product of eda_opmv, (3.16) or
// (3.2), for callers that cannot allocate device memory (work under HIP
// graph capture, tight serving loops, harnesses that forbid allocation).
//
// The product's scratch -- the row-chunk partials of P^T V, Y = P^T V, the
// column-group partials of the core product and Z = C Y -- lives in one
// file-scope device array of kScratchBytes per device instead of the
// handle's workspaces.  Its device address is looked up once per device by
// hipGetSymbolAddress (at eda_create, with that device current) and only
// that address is passed to the kernels.  Every call on a device shares the
// array: calls that overlap on one device (two streams, two threads) race.
// Nothing in it needs clearing: every kernel writes all the entries the next
// one reads.  The launches and their order are those of eda_opmv, so the
// two entry points give the same bits.
#include <hip/hip_runtime.h>

#include <mutex>

#include "host_internal.h"

using namespace eda;

namespace {

constexpr size_t kScratchBytes = (size_t)32 << 20;  // 32 MiB on every device the library runs on
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

}  // namespace

namespace eda {

hipError_t noalloc_init_device(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> g(g_mu);
  if (g_scratch[device] != nullptr) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return e;
  }
  g_scratch[device] = p;
  return hipSuccess;
}

}  // namespace eda

extern "C" eda_status eda_opmv_noalloc(eda_handle h, eda_form form, int64_t b, const void* V,
                                       int64_t ldv, void* Out, int64_t ldo, eda_dtype vdtype,
                                       double* log_scale) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (form != EDA_FORM_LANCZOS_M && form != EDA_FORM_ARNOLDI_A)
    return fail(h, EDA_ERR_ARG, "unknown operator form");
  if (!h->prepared) return fail(h, EDA_ERR_STATE, "eda_prepare has not succeeded");
  STCHK(validate_block(h, b, V, ldv, Out, ldo, vdtype));
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, V, "V"));
  STCHK(check_dev_ptr(h, Out, "Out"));
  if (form == EDA_FORM_ARNOLDI_A && !h->ca_ready)
    return fail(h, EDA_ERR_STATE,
                "the Arnoldi core is built on first use: call eda_opmv with the Arnoldi form once");
  void* base = nullptr;
  {
    std::lock_guard<std::mutex> g(g_mu);
    if (h->device < kMaxDevices) base = g_scratch[h->device];
  }
  if (base == nullptr) {
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != h->device) {
      (void)hipGetLastError();
      return fail(h, EDA_ERR_STATE, "scratch of device %d not set up (make it current)", h->device);
    }
    const hipError_t e = noalloc_init_device(h->device);
    if (e != hipSuccess)
      return fail(h, EDA_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    std::lock_guard<std::mutex> g(g_mu);
    base = g_scratch[h->device];
  }
  const int64_t d = h->d, N = h->N;
  const DT pdt = dt_of(h->storage), vdt = dt_of(vdtype);
  const double* C = form == EDA_FORM_LANCZOS_M ? h->CM.d() : h->CA.d();
  const bool split = core_split(N, b, C, N);
  const int64_t chunks = tn_chunks(d, N, b);
  const size_t part_b = align256((size_t)chunks * N * b * 8);
  const size_t y_b = align256((size_t)N * b * 8);
  const size_t z_b = align256((size_t)N * b * 8);
  const size_t zp_b = split ? align256((size_t)nn_split_groups(N) * N * b * 8) : 0;
  const bool nsplit = narrow_split(pdt, vdt, vdt, b, h->ldp);
  const size_t np_b = nsplit ? align256((size_t)nn_narrow_split_groups(d, N) * d * 8 * 4) : 0;
  const size_t need = part_b + y_b + z_b + zp_b + np_b;
  if (need > kScratchBytes)
    return fail(h, EDA_ERR_ARG,
                "this product needs %zu bytes of scratch, more than the %zu of eda_opmv_noalloc "
                "(use eda_opmv, or fewer columns)",
                need, kScratchBytes);
  char* sp = (char*)base;
  double* part = (double*)sp;
  double* ysm = (double*)(sp + part_b);
  double* zsm = (double*)(sp + part_b + y_b);
  double* zpart = (double*)(sp + part_b + y_b + z_b);
  float* npart = (float*)(sp + part_b + y_b + z_b + zp_b);
  const double* sc = (pdt == DT::FP8) ? h->pscale.d() : nullptr;
  hipStream_t s = h->stream;
  HIPCHK(launch_tn_partial(d, N, b, h->P.p, pdt, h->ldp, V, vdt, ldv, part, chunks, nullptr, s, sc));
  HIPCHK(launch_reduce_partials(chunks, N, b, part, 0.0, 0.0, nullptr, 0, 1.0, ysm, b, nullptr, s));
  if (split)
    HIPCHK(launch_nn_split(N, b, C, N, ysm, b, zpart, zsm, b, s));
  else
    HIPCHK(launch_nn(N, N, b, C, DT::F64, N, ysm, b, 0.0, nullptr, DT::F64, 0, zsm, DT::F64, b,
                     nullptr, s, true));
  // the second pass as eda_opmv takes it
  hipError_t e2 = hipErrorInvalidValue;
  if (nsplit)
    e2 = launch_nn_narrow_split(d, N, b, h->P.p, pdt, h->ldp, zsm, b, h->alphaB, nullptr, V, vdt,
                                ldv, Out, vdt, ldo, sc, npart, s);
  if (e2 == hipErrorInvalidValue)
    HIPCHK(launch_nn(d, N, b, h->P.p, pdt, h->ldp, zsm, b, h->alphaB, V, vdt, ldv, Out, vdt, ldo,
                     nullptr, s, false, nullptr, sc));
  else if (e2 != hipSuccess)
    return fail(h, EDA_ERR_HIP, "launch_nn_narrow_split failed: %s", hipGetErrorString(e2));
  if (log_scale != nullptr) *log_scale = h->shiftB;
  return EDA_OK;
}
