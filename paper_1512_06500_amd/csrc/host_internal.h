// Internal state and helpers shared by the host-side sources of libeda
// (eda_api.cpp: handle, preparation, products; eda_solve.cpp: the solver).
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "common.h"
#include "eda.h"

namespace eda {

struct Buf {
  void* p = nullptr;
  size_t cap = 0;
  double* d() const { return (double*)p; }
  float* f() const { return (float*)p; }
  int* i() const { return (int*)p; }
  char* c() const { return (char*)p; }
};

struct BatchState;  // eda_solve_batched workspaces (eda_batched.cpp)

struct StepGraph {  // captured block step (product and orthonormalisation)
  int64_t m;
  int cur;
  bool repair;
  hipGraphExec_t op, rest;
};

struct CoreEntry {
  int which = -1;
  double c = 0.0;
  double shift = 0.0;
  Buf buf;
};

constexpr double kU64 = 1.1102230246251565e-16;  // 2^-53

}  // namespace eda

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
  eda::Buf P;    // P = [H_W H_B] in storage precision (ld ldp)
  eda::Buf P64;  // float64 master of P when storage is not float64
  eda::Buf G, eigW, eigZ, nsbuf, Gh, Gm, GBs, CM, CA, T1, T2, T3, T4, fw, polyws, normbuf;
  eda::Buf gws;  // split partial tiles of the symmetric GEMMs on the handle's stream
  double shiftB = 0.0, alphaB = 1.0;
  eda::Buf alphaB_dev;  // alphaB on the device, read by captured steps
  eda::Buf pscale;      // FP8 storage: column j of P is pscale[j] times its FP8 copy
  eda::Buf dir[10];     // workspaces of eda_solve_direct
  eda::Buf warm;        // start block of a float64 continuation (and its mixing matrix)
  eda::Buf af[10];      // workspaces of the Arnoldi-form solve
  eda::Buf nnp[2];      // projections of the classifier (training, testing)
  double normW = 0.0;   // ||H_W^T H_W||_1
  bool w_eig = false;   // eigenpairs of H_W^T H_W available
  bool ca_ready = false;  // Arnoldi core C_A built for the current preparation
  std::vector<double> hwW, hwB;
  double t_prepare_ms = 0.0;
  bool prep_time_pending = false;  // prep_ev[0..1] recorded, t_prepare_ms not yet read
  // pinned host scalars of the preparation (non-finite flag, ||G_WW||_1,
  // eigenvalues of G_BB and of G_WW), read back without a blocking copy
  void* pin = nullptr;
  size_t pin_cap = 0;
  // prep_ev: [0] start, [1] end of the preparation, [2] Gram ready (the
  // second stream starts eig(H_B^T H_B)), [3] that eigensolve copied out
  hipEvent_t prep_ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool prep_wbyeig = false;
  bool prep_overlap = false;  // eig(H_B^T H_B) on the second stream beside the W-cores
  // the W-core polynomial may read its spectral bound back to the host (a
  // drain of the stream); off for the per-problem handles of a batch, whose
  // preparations are enqueued back to back
  bool poly_readback = true;

  // workspaces
  eda::Buf part, Ysm, Zsm, syev_work, offs, flags, mask;
  eda::Buf zpart;  // column-group partials of the split core product Z = C Y
  eda::Buf npart;  // float32 column-group partials of the narrow second pass
  std::vector<eda::CoreEntry> cores;

  // solver
  eda::Buf Q[2], H[2], Wb, T, wT, S, Sd, hz, Gs, Rinv, R1, Yb, MYb, dtheta, dres, refine;
  // P^T Q of the live basis (row-major N x (mmax + b)), float64 storage only:
  // filled block by block by the products of the Krylov phase
  eda::Buf PQ[2];

  // captured block steps of the current solver configuration
  std::vector<eda::StepGraph> graphs;
  uint64_t graph_sig = 0;
  hipStream_t cap = nullptr;

  // second stream for Rayleigh-Ritz checks that overlap the next block steps
  hipStream_t aux = nullptr;
  hipEvent_t ev_main = nullptr, ev_rr = nullptr;
  double* rr_pin = nullptr;  // pinned readback of Ritz values and estimates
  size_t rr_pin_cap = 0;

  // batched solver
  eda::BatchState* batch = nullptr;
};

namespace eda {

eda_status fail(eda_handle h, eda_status s, const char* fmt, ...);
eda_status ensure(eda_handle h, Buf& b, size_t bytes);
void release(Buf& b);
eda_status need_device(eda_handle h);
eda_status check_dev_ptr(eda_handle h, const void* p, const char* name);

inline size_t dsize(eda_dtype t) {
  return t == EDA_F64 ? 8 : (t == EDA_F32 ? 4 : (t == EDA_BF16 ? 2 : 1));
}
inline DT dt_of(eda_dtype t) {
  return t == EDA_F64 ? DT::F64 : (t == EDA_F32 ? DT::F32 : (t == EDA_BF16 ? DT::BF16 : DT::FP8));
}
inline size_t dt_size(DT t) {
  return t == DT::F64 ? 8 : (t == DT::F32 ? 4 : (t == DT::BF16 ? 2 : 1));
}
inline int64_t round_up(int64_t x, int64_t m) { return ((x + m - 1) / m) * m; }

// eda_prepare in two halves: prepare_begin validates and enqueues every
// kernel up to the small eigensolves, with the scalars the host needs copied
// asynchronously into pinned memory; after the stream has drained,
// prepare_end reads them (non-finite check, spectral shift) and enqueues the
// core construction.  Neither half blocks the host, except that prepare_end
// waits once for the spectral bound of the W-core polynomial on a handle
// with poly_readback set (the per-problem handles of a batch have it off).
// With `overlap`, eig(H_B^T H_B) runs on the second stream so that
// prepare_end can build the W-cores (which need only ||H_W^T H_W||_1) while
// it runs; the caller then needs to drain only the main stream before
// prepare_end.
eda_status prepare_begin(eda_handle h, int64_t d, int64_t n, int64_t k, const double* H_W,
                         int64_t ldw, const double* H_B, int64_t ldb, eda_dtype storage,
                         bool overlap = false);
eda_status prepare_end(eda_handle h);
// Duration of the last eda_prepare from its events, read on first use (by
// then the preparation has normally finished: nothing waits for it at the
// end of eda_prepare).
double prepare_time_ms(eda_handle h);
void destroy_batch_state(eda_handle h);
void release_graphs(eda_handle h);

// x = exp(-S_W/2) y for t columns, orthonormalised (Cholesky QR twice,
// scratch ld ldw) and sign-fixed.  With `ysm_ready`, h->Ysm already holds
// P^T Y from the product just taken of the same Y (float64 master), and
// only the second pass runs.
eda_status back_transform(eda_handle h, int64_t t, const double* Y, int64_t ldy, double* X,
                          int64_t ldx, int64_t ldw, bool ysm_ready = false);
// Columns of X (d x t) orthonormalised in column order by Cholesky QR run
// twice (scratch with leading dimension ldw in h->Yb) and sign-fixed.
eda_status orthonormalise(eda_handle h, int64_t t, double* X, int64_t ldx, int64_t ldw);
// The Arnoldi core C_A of the current preparation, built on first use (the
// Lanczos form does not need it).
eda_status ensure_arnoldi_core(eda_handle h);
// Core of exp(c S_W) without shift (exp(c S_W) = I + H_W C H_W^T), n x n.
eda_status build_w_core(eda_handle h, double c, double* out);
// Measures the candidate launch shapes of the product passes for a d x N
// matrix in `storage` and b float64 columns and records the fastest
// (eda_tune.cpp).  Outputs may be null.
eda_status autotune_shapes(eda_handle h, int64_t d, int64_t N, int64_t b, eda_dtype storage,
                           int32_t* tn_out, int32_t* nn_out, double* us_out);
// eda_solve for the Arnoldi form (eda_aform.cpp); arguments already checked.
eda_status solve_aform(eda_handle h, int32_t t, double tol, const eda_solve_opts& o,
                       double* ritz, double* ritz_log, double* X, int64_t ldx, double* resid,
                       eda_info* info);
// Checks of an operand block V and output block Out of b columns (eda_expmv,
// eda_opmv): shapes, types, leading dimensions, no overlap.
eda_status validate_block(eda_handle h, int64_t b, const void* V, int64_t ldv, const void* Out,
                          int64_t ldo, eda_dtype vdtype);
// Whether the core product Z = C Y of a product over Nc columns is split
// over column groups of C (launch_nn_split) rather than one streaming launch.
inline bool core_split(int64_t Nc, int64_t b, const double* C, int64_t ldc) {
  return Nc >= 1024 && b <= 16 && ldc % 2 == 0 && ((uintptr_t)C % 16) == 0;
}
// Makes the float64 master the storage copy of a narrow preparation (the
// Gram and the cores already come from the float64 factors, so nothing is
// rebuilt); a float64 preparation is left as it is.
eda_status promote_storage_f64(eda_handle h);
// Start block of a float64 continuation from a Ritz block Y (d x t, ld ldy):
// Y G with a fixed pseudo-random t x b mixing G when t >= b, else Y followed
// by b - t Gaussian columns.  Written to h->warm (d x b, ld d).
eda_status warm_start_block(eda_handle h, int64_t d, int64_t t, int64_t b, const double* Y,
                            int64_t ldy, uint64_t seed, double** V, int64_t* ldv);
// One Cholesky QR pass: G = X^T X, Xout = X R^{-1}.  Optionally records R
// (combined with Rprev) and raises the repair flag.
eda_status cholqr_pass(eda_handle h, int64_t d, int64_t cols, const void* X, DT xdt, int64_t ldx,
                       void* Xout, int64_t ldxo, const double* Rprev, double* Rout, int64_t ldro,
                       const double* hcol, int64_t mrows, int64_t ldhc, const int* gate,
                       int* flag);
// One classical Gram-Schmidt pass of W (b columns) against Q[:, 0:m]:
//   h = Q^T W (accumulated into Hcol when given),  W -= Q h.
eda_status cgs_pass(eda_handle h, int64_t d, int64_t m, const void* Q, DT qdt, int64_t ldq,
                    void* W, int64_t ldw, int64_t b, double* Hcol, int64_t ldh, double beta,
                    const int* gate);
// float64 Rayleigh-Ritz on the w columns of B (with MB = M B): the top t
// Ritz vectors go to Y = B S_t and MY = MB S_t, the Ritz values (descending)
// to dtheta.  Uses the workspaces T, S, wT, Sd with leading dimension mm.
eda_status rr_block(eda_handle h, int64_t d, int64_t ld, int64_t w, int64_t t, int64_t mm,
                    const double* B, const double* MB, double* Y, double* MY);
// eda_solve by block Jacobi-Davidson (eda_jd.cpp); arguments already checked.
eda_status solve_jd(eda_handle h, int32_t t, double tol, const eda_solve_opts& o, double* ritz,
                    double* ritz_log, double* X, int64_t ldx, double* resid, eda_info* info);
// Whether the second pass of a product over a narrow factor takes the
// column-split kernel (launch_nn_narrow_split) with float32 partial rows.
inline bool narrow_split(DT pdt, DT vdt, DT odt, int64_t b, int64_t ldp) {
  return (pdt == DT::BF16 || pdt == DT::FP8) && (vdt == DT::F32 || vdt == DT::BF16) && b <= 8 &&
         vdt == odt && ldp % 8 == 0;
}
// Looks up, once per device, the device address of the scratch array of
// eda_opmv_noalloc (eda_noalloc.hip); the device must be current.
hipError_t noalloc_init_device(int device);
// Low-rank exponential apply on columns [c0, c0+Nc) of P (the storage copy,
// or the float64 master when `master`):  Out = alpha V + P_c C P_c^T V.
eda_status expop(eda_handle h, bool master, int64_t c0, int64_t Nc, const double* C,
                 int64_t ldc, double alpha, int64_t b, const void* V, DT vdt, int64_t ldv,
                 void* Out, DT odt, int64_t ldo, const double* alpha_p = nullptr);
// Its two halves: h->Ysm = P_c^T V (row-major, Nc x b), then
// Out = alpha V + P_c (C Ysm).  The second half may take a leading block of
// columns of an earlier first half (Nc no larger, same b, same V).
// (ysm, ldy): where P_c^T V goes (row-major), h->Ysm with ld b by default.
eda_status expop_first(eda_handle h, bool master, int64_t c0, int64_t Nc, int64_t b,
                       const void* V, DT vdt, int64_t ldv, double* ysm = nullptr,
                       int64_t ldy = 0);
eda_status expop_second(eda_handle h, bool master, int64_t c0, int64_t Nc, const double* C,
                        int64_t ldc, double alpha, int64_t b, const void* V, DT vdt,
                        int64_t ldv, void* Out, DT odt, int64_t ldo,
                        const double* alpha_p = nullptr, const double* ysm = nullptr,
                        int64_t ldy = 0);

}  // namespace eda

#define HIPCHK(x)                                                                       \
  do {                                                                                  \
    hipError_t e_ = (x);                                                                \
    if (e_ != hipSuccess)                                                               \
      return ::eda::fail(h, EDA_ERR_HIP, "%s failed: %s", #x, hipGetErrorString(e_));   \
  } while (0)

#define STCHK(x)                 \
  do {                           \
    eda_status s_ = (x);         \
    if (s_ != EDA_OK) return s_; \
  } while (0)
