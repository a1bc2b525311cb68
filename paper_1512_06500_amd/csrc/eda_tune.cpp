// Autotuner of the streaming kernels' launch shapes.
//
// The two passes of the low-rank exponential product (tn: P^T V over row
// chunks, nn: alpha V + P Z) each have a few launch shapes: tn the number of
// 64-row steps per wave (which fixes how many row chunks, and so how many
// partial sums, a product has), nn the rows per workgroup and the loads per
// batch.  Their size heuristics are replaced, per shape class
// (ceil(log2 d), ceil(log2 N), entry size), by the fastest shape measured on
// the device.  Results live in a process-wide table, and in the text file
// named by EDA_TUNE_CACHE when that is set (read once, rewritten after every
// tuning), one entry per line: "tn|nn <log2 d> <log2 N> <entry bytes> <choice>".
// Every shape computes the same products; only the order of their partial
// sums changes.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "host_internal.h"

using namespace eda;

namespace {

std::mutex g_mu;
std::map<uint64_t, int> g_table;
bool g_loaded = false;
std::atomic<bool> g_any{false};

int clog2(int64_t x) {
  int l = 0;
  while (l < 62 && (int64_t(1) << l) < x) ++l;
  return l;
}

uint64_t make_key(int kind, int dl, int ml, int es) {
  return ((uint64_t)kind << 48) | ((uint64_t)dl << 32) | ((uint64_t)ml << 16) | (uint64_t)es;
}

void load_locked() {
  if (g_loaded) return;
  g_loaded = true;
  const char* path = std::getenv("EDA_TUNE_CACHE");
  if (path == nullptr) return;
  FILE* f = std::fopen(path, "r");
  if (f == nullptr) return;
  char kind[8];
  int dl, ml, es, v;
  while (std::fscanf(f, "%7s %d %d %d %d", kind, &dl, &ml, &es, &v) == 5) {
    const bool tn = std::strcmp(kind, "tn") == 0, nn = std::strcmp(kind, "nn") == 0;
    if ((!tn && !nn) || dl < 0 || dl > 62 || ml < 0 || ml > 62 || es < 0 || es > 8) continue;
    if (tn && v != 1 && v != 2 && v != 4 && v != 8) continue;
    if (nn && (v < 0 || v >= kNnConfigs)) continue;
    g_table[make_key(tn ? 0 : 1, dl, ml, es)] = v;
  }
  std::fclose(f);
  if (!g_table.empty()) g_any = true;
}

void save_locked() {
  const char* path = std::getenv("EDA_TUNE_CACHE");
  if (path == nullptr) return;
  FILE* f = std::fopen(path, "w");
  if (f == nullptr) return;
  for (const auto& e : g_table) {
    const int kind = (int)(e.first >> 48), dl = (int)((e.first >> 32) & 0xffff);
    const int ml = (int)((e.first >> 16) & 0xffff), es = (int)(e.first & 0xffff);
    std::fprintf(f, "%s %d %d %d %d\n", kind == 0 ? "tn" : "nn", dl, ml, es, e.second);
  }
  std::fclose(f);
}

}  // namespace

namespace eda {

int tune_get(TuneKind kind, int64_t d, int64_t m, int esize) {
  if (!g_any.load(std::memory_order_acquire)) {
    std::lock_guard<std::mutex> g(g_mu);
    load_locked();
    if (g_table.empty()) return -1;
  }
  std::lock_guard<std::mutex> g(g_mu);
  const auto it = g_table.find(make_key((int)kind, clog2(d), clog2(m), esize));
  return it == g_table.end() ? -1 : it->second;
}

void tune_set(TuneKind kind, int64_t d, int64_t m, int esize, int value) {
  std::lock_guard<std::mutex> g(g_mu);
  load_locked();
  g_table[make_key((int)kind, clog2(d), clog2(m), esize)] = value;
  g_any = true;
}

// Measures every candidate shape of the product passes for a d x N matrix of
// the given storage and a block of b float64 columns, keeps the fastest.
eda_status autotune_shapes(eda_handle h, int64_t d, int64_t N, int64_t b, eda_dtype storage,
                           int32_t* tn_out, int32_t* nn_out, double* us_out) {
  const int64_t ld = round_up(d, 64);
  const size_t es = dsize(storage);
  const DT adt = dt_of(storage);
  hipStream_t s = h->stream;
  Buf A, V, Z, O, part;
  eda_status st = EDA_OK;
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    release(A);
    release(V);
    release(Z);
    release(O);
    release(part);
  };
  if ((st = ensure(h, A, ld * N * es)) != EDA_OK || (st = ensure(h, V, ld * b * 8)) != EDA_OK ||
      (st = ensure(h, Z, N * b * 8)) != EDA_OK || (st = ensure(h, O, ld * b * 8)) != EDA_OK) {
    cleanup();
    return st;
  }
  // contents do not change the timings: zero operands (zero is finite in
  // every storage type)
  hipError_t e = launch_fill_i32((int64_t)(ld * N * es / 4), 0, A.i(), s);
  if (e == hipSuccess) e = launch_fill(ld * b, 0.0, V.d(), s);
  if (e == hipSuccess) e = launch_fill(N * b, 0.0, Z.d(), s);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  auto timed = [&](auto launch, double* us) -> hipError_t {
    hipError_t r = hipSuccess;
    for (int i = 0; i < 2 && r == hipSuccess; ++i) r = launch();
    if (r == hipSuccess) r = hipEventRecord(e0, s);
    for (int i = 0; i < 5 && r == hipSuccess; ++i) r = launch();
    if (r == hipSuccess) r = hipEventRecord(e1, s);
    if (r == hipSuccess) r = hipEventSynchronize(e1);
    float ms = 0.f;
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
    *us = 1e3 * ms / 5.0;
    return r;
  };
  // tn: 64-row steps per wave
  int best_s = -1;
  double best_tn = 1e30;
  for (int S : {1, 2, 4, 8}) {
    if (e != hipSuccess) break;
    tune_set(TuneKind::TnSteps, d, N, 0, S);
    const int64_t chunks = tn_chunks(d, N, b);
    if ((st = ensure(h, part, (size_t)chunks * N * b * 8)) != EDA_OK) break;
    double us = 0.0;
    e = timed([&]() {
      return launch_tn_partial(d, N, b, A.p, adt, ld, V.p, DT::F64, ld, part.d(), chunks, nullptr,
                               s);
    }, &us);
    if (e == hipSuccess && us < best_tn) {
      best_tn = us;
      best_s = S;
    }
  }
  if (best_s > 0) tune_set(TuneKind::TnSteps, d, N, 0, best_s);
  // nn: rows per workgroup and loads per batch (FP8 and bfloat16 storage use
  // the eight-rows-per-lane kernel, which has a single shape)
  int best_c = -1;
  double best_nn = 1e30;
  if (es == 8 || es == 4)
    for (int c = 0; c < kNnConfigs; ++c) {
      if (e != hipSuccess || st != EDA_OK) break;
      tune_set(TuneKind::NnTile, d, N, (int)es, c);
      double us = 0.0;
      e = timed([&]() {
        return launch_nn(d, N, b, A.p, adt, ld, Z.d(), b, 1.0, V.p, DT::F64, ld, O.p, DT::F64, ld,
                         nullptr, s);
      }, &us);
      if (e == hipSuccess && us < best_nn) {
        best_nn = us;
        best_c = c;
      }
    }
  if (best_c >= 0) tune_set(TuneKind::NnTile, d, N, (int)es, best_c);
  if (e0 != nullptr) (void)hipEventDestroy(e0);
  if (e1 != nullptr) (void)hipEventDestroy(e1);
  cleanup();
  if (st != EDA_OK) return st;
  if (e != hipSuccess) return fail(h, EDA_ERR_HIP, "autotune: %s", hipGetErrorString(e));
  {
    std::lock_guard<std::mutex> g(g_mu);
    save_locked();
  }
  if (tn_out != nullptr) *tn_out = best_s;
  if (nn_out != nullptr) *nn_out = best_c;
  if (us_out != nullptr) {
    us_out[0] = best_tn;
    us_out[1] = best_c >= 0 ? best_nn : 0.0;
  }
  return EDA_OK;
}

}  // namespace eda

extern "C" eda_status eda_autotune(eda_handle h, int64_t d, int64_t N, int32_t b,
                                   eda_dtype storage, int32_t* tn_steps, int32_t* nn_tile,
                                   double* us) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (d < 1 || N < 1 || b < 1 || b > 16)
    return fail(h, EDA_ERR_ARG, "need d >= 1, N >= 1, 1 <= b <= 16");
  if (storage != EDA_F64 && storage != EDA_F32 && storage != EDA_BF16 && storage != EDA_FP8_E4M3)
    return fail(h, EDA_ERR_ARG, "unknown storage type");
  STCHK(need_device(h));
  return autotune_shapes(h, d, N, b, storage, tn_steps, nn_tile, us);
}
