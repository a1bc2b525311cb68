// libeda host library, part 3: eda_solve_batched.
//
// Many independent problems (different d, n, k, t) solved together.  The
// algorithm per problem is exactly that of eda_solve (block Lanczos with
// thick restart on e^{-s} M, eqs. (3.13)-(3.16), float64 check and
// refinement, back-transform of eq. (3.14)); what changes is the execution:
// every kernel of a phase is launched once for all problems that take part
// in it, with per-problem arguments in a device array indexed by
// blockIdx.z.  The argument arrays of all launches up to the next host
// decision are gathered in pinned memory and sent in one copy, so a block
// Lanczos step of the whole batch costs the same number of launches as one
// problem's step.  Problems leave the launches when they converge.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#include "host_internal.h"

namespace eda {

// Pinned staging of argument arrays, flushed with one host-to-device copy
// ahead of the launches that read them.  Two host halves alternate so that
// the next batch of arguments can be written while the previous copy is in
// flight; the device side is a single buffer, reused in stream order.
struct ArgStage {
  char* host[2] = {nullptr, nullptr};
  char* dev = nullptr;
  size_t cap = 0, used = 0;
  int half = 0;
  hipEvent_t ev[2] = {nullptr, nullptr};
  bool ev_live[2] = {false, false};
  std::vector<std::function<hipError_t()>> pending;
};

struct BatchState {
  ArgStage st;
  void* arena = nullptr;
  size_t arena_cap = 0;
  double* hpin = nullptr;  // pinned readback of Ritz values and residuals
  size_t hpin_cap = 0;
  std::vector<eda_handle> subs;
  std::vector<hipEvent_t> ev;
};

void destroy_batch_state(eda_handle h) {
  BatchState* B = h->batch;
  if (B == nullptr) return;
  for (eda_handle s : B->subs) eda_destroy(s);
  for (int q = 0; q < 2; ++q) {
    if (B->st.host[q] != nullptr) (void)hipHostFree(B->st.host[q]);
    if (B->st.ev[q] != nullptr) (void)hipEventDestroy(B->st.ev[q]);
  }
  if (B->st.dev != nullptr) (void)hipFree(B->st.dev);
  if (B->arena != nullptr) (void)hipFree(B->arena);
  if (B->hpin != nullptr) (void)hipHostFree(B->hpin);
  for (hipEvent_t e : B->ev) (void)hipEventDestroy(e);
  delete B;
  h->batch = nullptr;
}

}  // namespace eda

using namespace eda;

namespace {

constexpr size_t kStageBytes = size_t(4) << 20;

double unit_roundoff(DT t) {
  switch (t) {
    case DT::F64: return 0x1.0p-53;
    case DT::F32: return 0x1.0p-24;
    case DT::BF16: return 0x1.0p-8;
    default: return 0x1.0p-4;  // FP8 E4M3
  }
}

// Executes the recorded launches: one copy of the staged arguments, then
// the launches in order.
eda_status stage_run(eda_handle h) {
  ArgStage& st = h->batch->st;
  if (st.used > 0) {
    HIPCHK(hipMemcpyAsync(st.dev, st.host[st.half], st.used, hipMemcpyHostToDevice, h->stream));
    HIPCHK(hipEventRecord(st.ev[st.half], h->stream));
    st.ev_live[st.half] = true;
  }
  for (auto& f : st.pending) {
    const hipError_t e = f();
    if (e != hipSuccess) {
      st.pending.clear();
      return fail(h, EDA_ERR_HIP, "batched launch failed: %s", hipGetErrorString(e));
    }
  }
  st.pending.clear();
  st.used = 0;
  st.half ^= 1;
  if (st.ev_live[st.half]) {  // the half about to be rewritten must have been copied
    HIPCHK(hipEventSynchronize(st.ev[st.half]));
    st.ev_live[st.half] = false;
  }
  return EDA_OK;
}

// Records one multi launch; `launch(count, host, dev)` issues it.
template <class A, class L>
eda_status push(eda_handle h, std::vector<A>&& v, L launch) {
  if (v.empty()) return EDA_OK;
  ArgStage& st = h->batch->st;
  const A* dv = nullptr;
  if (v.size() > 1) {
    const size_t bytes = v.size() * sizeof(A);
    if (bytes > st.cap) return fail(h, EDA_ERR_ARG, "argument array of %zu bytes too large", bytes);
    size_t off = (st.used + 15) & ~size_t(15);
    if (off + bytes > st.cap) {
      STCHK(stage_run(h));
      off = 0;
    }
    std::memcpy(st.host[st.half] + off, v.data(), bytes);
    dv = (const A*)(st.dev + off);
    st.used = off + bytes;
  }
  st.pending.push_back([v = std::move(v), dv, launch]() {
    return launch((int)v.size(), v.data(), dv);
  });
  return EDA_OK;
}

// Any stream operation in launch order (event records, copies).
eda_status push_op(eda_handle h, std::function<hipError_t()> f) {
  h->batch->st.pending.push_back(std::move(f));
  return EDA_OK;
}

struct BP {
  eda_handle sub = nullptr;  // preparation of this problem
  const eda_problem* pr = nullptr;
  int32_t t = 0;
  double tol = 0.0;
  int64_t d = 0, n = 0, k = 0, N = 0, ldq = 0, mmax = 0, ldh = 0, kk = 0, wz = 0, mm = 0, bt = 0;
  // workspace
  char* Q[2] = {nullptr, nullptr};
  double* H[2] = {nullptr, nullptr};
  char* W = nullptr;
  double *Yb = nullptr, *T = nullptr, *S = nullptr, *wT = nullptr, *Sd = nullptr;
  double *part = nullptr, *Ysm = nullptr, *Zsm = nullptr, *hz = nullptr, *Gs = nullptr;
  double *Rinv = nullptr, *R1 = nullptr, *dtheta = nullptr, *dres = nullptr, *syw = nullptr;
  double* refine = nullptr;
  int *flags = nullptr, *mask = nullptr;
  double* hth = nullptr;  // pinned readback slots
  double* hre = nullptr;
  int* hfl = nullptr;
  // state
  int cur = 0, cb = 0;
  int64_t m = 0, iters = 0, restarts = 0, m_rr = 0, passes = 0, ops = 0, op_calls = 0;
  double bytes = 0.0, t_op_ms = 0.0;
  bool active = true, kconv = false, converged = false, floor_limited = false;
  int flags_out = 0;
  std::vector<double> theta, est;
  double* XB[2] = {nullptr, nullptr};
  double* MB[2] = {nullptr, nullptr};
  char* Qc(int64_t j, size_t qs) const { return Q[cur] + (size_t)j * ldq * qs; }
};

struct Engine {
  eda_handle h;
  std::vector<BP> P;
  int64_t b = 8, check_every = 2, max_iter = 4000, max_refine = 2;
  DT qdt = DT::F64, sdt = DT::F64;
  size_t qs = 8;
  bool mixed = false;
  double u_lo = 0x1.0p-53;
  eda_resmode resmode = EDA_RES_REL_THETA;
  int64_t mm_all = 0;  // largest Rayleigh-Ritz dimension (eigensolver work size)
  uint64_t seed = 0;   // problem p draws its start block from seed + p
};

// ---- multi-launch helpers (one entry per listed problem) --------------------

template <class F>
eda_status m_tn(Engine& E, const std::vector<int>& ps, DT adt, DT bdt, F f) {
  std::vector<TnArgs> v;
  int64_t dmax = 0, mmax = 0;
  for (int i : ps) {
    v.push_back(f(E.P[i]));
    dmax = std::max(dmax, v.back().d);
    mmax = std::max(mmax, v.back().m);
  }
  for (auto& a : v) a.chunks = tn_chunks_for(a.d, dmax, mmax);
  return push(E.h, std::move(v), [adt, bdt, s = E.h->stream](int c, const TnArgs* hh,
                                                             const TnArgs* dd) {
    return launch_tn_multi(c, hh, dd, adt, bdt, s);
  });
}

template <class F>
eda_status m_reduce(Engine& E, const std::vector<int>& ps, F f) {
  std::vector<ReduceArgs> v;
  for (int i : ps) v.push_back(f(E.P[i]));
  return push(E.h, std::move(v), [s = E.h->stream](int c, const ReduceArgs* hh,
                                                    const ReduceArgs* dd) {
    return launch_reduce_multi(c, hh, dd, s);
  });
}

template <class F>
eda_status m_nn(Engine& E, const std::vector<int>& ps, DT adt, DT vdt, DT odt, F f) {
  std::vector<NnArgs> v;
  for (int i : ps) v.push_back(f(E.P[i]));
  return push(E.h, std::move(v), [adt, vdt, odt, s = E.h->stream](int c, const NnArgs* hh,
                                                                   const NnArgs* dd) {
    return launch_nn_multi(c, hh, dd, adt, vdt, odt, s);
  });
}

#define M_SIMPLE(name, Args, launcher)                                                    \
  template <class F>                                                                      \
  eda_status name(Engine& E, const std::vector<int>& ps, F f) {                           \
    std::vector<Args> v;                                                                  \
    for (int i : ps) v.push_back(f(E.P[i]));                                              \
    return push(E.h, std::move(v), [s = E.h->stream](int c, const Args* hh, const Args* dd) { \
      return launcher(c, hh, dd, s);                                                      \
    });                                                                                   \
  }
M_SIMPLE(m_chol, CholArgs, launch_chol_multi)
M_SIMPLE(m_pchol, PcholArgs, launch_pchol_multi)
M_SIMPLE(m_randn, RandnArgs, launch_randn_multi)
M_SIMPLE(m_fill, FillArgs, launch_fill_multi)
M_SIMPLE(m_fill_i32, FillI32Args, launch_fill_i32_multi)
M_SIMPLE(m_sym, SymArgs, launch_symmetrize_multi)
M_SIMPLE(m_ritzest, RitzEstArgs, launch_ritz_estimates_multi)
M_SIMPLE(m_gather, GatherArgs, launch_gather_desc_multi)
M_SIMPLE(m_setdiag, SetDiagArgs, launch_set_diag_multi)
M_SIMPLE(m_coupling, CouplingArgs, launch_restart_coupling_multi)
M_SIMPLE(m_resid, ResidArgs, launch_ritz_residual_multi)
M_SIMPLE(m_desc, DescArgs, launch_desc_values_multi)
M_SIMPLE(m_sign, SignArgs, launch_sign_fix_multi)
M_SIMPLE(m_fold, FlagArgs, launch_flag_fold_multi)
M_SIMPLE(m_syev, SyevArgs, launch_syev_multi)
#undef M_SIMPLE

template <class F>
eda_status m_copy(Engine& E, const std::vector<int>& ps, DT sdt, DT ddt, F f) {
  std::vector<Copy2dArgs> v;
  for (int i : ps) v.push_back(f(E.P[i]));
  return push(E.h, std::move(v), [sdt, ddt, s = E.h->stream](int c, const Copy2dArgs* hh,
                                                             const Copy2dArgs* dd) {
    return launch_copy2d_multi(c, hh, dd, sdt, ddt, s);
  });
}

template <class F>
eda_status m_mrandn(Engine& E, const std::vector<int>& ps, DT qdt, F f) {
  std::vector<MaskedRandnArgs> v;
  for (int i : ps) v.push_back(f(E.P[i]));
  return push(E.h, std::move(v), [qdt, s = E.h->stream](int c, const MaskedRandnArgs* hh,
                                                        const MaskedRandnArgs* dd) {
    return launch_masked_randn_multi(c, hh, dd, qdt, s);
  });
}

// X (cols columns, xdt) -> Xout = X R^{-1}, R from G = X^T X (Cholesky QR pass).
// X/Xout/ld given per problem by f: returns {X, ldx, Xout, ldxo, cols, Rprev, Rout, ldro, flag, gate}.
struct QRSite {
  const void* X;
  int64_t ldx;
  void* Xout;
  int64_t ldxo, cols;
  const double* Rprev;
  double* Rout;
  int64_t ldro;
  int* flag;
  const int* gate;
};

template <class F>
eda_status m_cholqr(Engine& E, const std::vector<int>& ps, DT xdt, F f) {
  std::vector<QRSite> sites;
  for (int i : ps) sites.push_back(f(E.P[i]));
  // tn (X^T X)
  {
    std::vector<TnArgs> v;
    int64_t dmax = 0, mmax = 0;
    for (size_t q = 0; q < ps.size(); ++q) {
      BP& p = E.P[ps[q]];
      const QRSite& s = sites[q];
      v.push_back(TnArgs{p.d, s.cols, s.cols, s.ldx, s.ldx, 0, s.X, s.X, p.part, s.gate});
      dmax = std::max(dmax, p.d);
      mmax = std::max(mmax, s.cols);
    }
    for (auto& a : v) a.chunks = tn_chunks_for(a.d, dmax, mmax);
    std::vector<ReduceArgs> r;
    std::vector<CholArgs> c;
    std::vector<NnArgs> n;
    for (size_t q = 0; q < ps.size(); ++q) {
      BP& p = E.P[ps[q]];
      const QRSite& s = sites[q];
      r.push_back(ReduceArgs{v[q].chunks, s.cols, s.cols, s.cols, 0, p.part, 1.0, 0.0, 0.0, p.Gs,
                             nullptr, s.gate});
      c.push_back(CholArgs{s.cols, s.cols, s.cols, s.cols, s.ldro, 0, 0, p.Gs, p.Rinv, s.Rprev,
                           s.Rout, nullptr, 1e-4, s.flag, s.gate});
      n.push_back(NnArgs{p.d, s.cols, s.cols, s.ldx, s.cols, s.ldx, s.ldxo, s.X, p.Rinv, 0.0,
                         nullptr, s.Xout, 0, s.gate});
    }
    eda_handle h = E.h;
    hipStream_t st = h->stream;
    STCHK(push(h, std::move(v), [xdt, st](int cc, const TnArgs* hh, const TnArgs* dd) {
      return launch_tn_multi(cc, hh, dd, xdt, xdt, st);
    }));
    STCHK(push(h, std::move(r), [st](int cc, const ReduceArgs* hh, const ReduceArgs* dd) {
      return launch_reduce_multi(cc, hh, dd, st);
    }));
    STCHK(push(h, std::move(c), [st](int cc, const CholArgs* hh, const CholArgs* dd) {
      return launch_chol_multi(cc, hh, dd, st);
    }));
    STCHK(push(h, std::move(n), [xdt, st](int cc, const NnArgs* hh, const NnArgs* dd) {
      return launch_nn_multi(cc, hh, dd, xdt, xdt, xdt, st);
    }));
  }
  return EDA_OK;
}

// One classical Gram-Schmidt pass of W (nb columns) against Q (m columns):
// h = Q^T W (accumulated into Hcol when given), W -= Q h.
struct CGSSite {
  const void* Q;
  int64_t ldq, m;
  void* W;
  int64_t ldw, nb;
  double* Hcol;
  int64_t ldh;
  double beta;
  const int* gate;
};

template <class F>
eda_status m_cgs(Engine& E, const std::vector<int>& ps, DT qdt, F f) {
  std::vector<CGSSite> sites;
  for (int i : ps) sites.push_back(f(E.P[i]));
  std::vector<TnArgs> v;
  int64_t dmax = 0, mmax = 0;
  for (size_t q = 0; q < ps.size(); ++q) {
    BP& p = E.P[ps[q]];
    const CGSSite& s = sites[q];
    v.push_back(TnArgs{p.d, s.m, s.nb, s.ldq, s.ldw, 0, s.Q, s.W, p.part, s.gate});
    dmax = std::max(dmax, p.d);
    mmax = std::max(mmax, s.m);
  }
  for (auto& a : v) a.chunks = tn_chunks_for(a.d, dmax, mmax);
  std::vector<ReduceArgs> r;
  std::vector<NnArgs> n;
  for (size_t q = 0; q < ps.size(); ++q) {
    BP& p = E.P[ps[q]];
    const CGSSite& s = sites[q];
    r.push_back(ReduceArgs{v[q].chunks, s.m, s.nb, s.ldh, s.nb, p.part, 1.0, s.beta, -1.0, s.Hcol,
                           p.hz, s.gate});
    n.push_back(NnArgs{p.d, s.m, s.nb, s.ldq, s.nb, s.ldw, s.ldw, s.Q, p.hz, 1.0, s.W, s.W, 0,
                       s.gate});
  }
  eda_handle h = E.h;
  hipStream_t st = h->stream;
  STCHK(push(h, std::move(v), [qdt, st](int cc, const TnArgs* hh, const TnArgs* dd) {
    return launch_tn_multi(cc, hh, dd, qdt, qdt, st);
  }));
  STCHK(push(h, std::move(r), [st](int cc, const ReduceArgs* hh, const ReduceArgs* dd) {
    return launch_reduce_multi(cc, hh, dd, st);
  }));
  STCHK(push(h, std::move(n), [qdt, st](int cc, const NnArgs* hh, const NnArgs* dd) {
    return launch_nn_multi(cc, hh, dd, qdt, qdt, qdt, st);
  }));
  return EDA_OK;
}

// Exponential product Out = alpha V + P_c C P_c^T V for each problem, with
// P the storage copy (master = false) or the float64 master.
struct OpSite {
  bool master;
  int64_t c0, Nc;
  const double* C;
  int64_t ldc;
  double alpha;
  int64_t nb;
  const void* V;
  int64_t ldv;
  void* Out;
  int64_t ldo;
};

template <class F>
eda_status m_expop(Engine& E, const std::vector<int>& ps, DT vdt, DT odt, F f) {
  if (ps.empty()) return EDA_OK;
  std::vector<OpSite> sites;
  for (int i : ps) sites.push_back(f(E.P[i]));
  const bool master = sites[0].master;
  DT pdt = master ? DT::F64 : E.sdt;
  std::vector<TnArgs> v;
  int64_t dmax = 0, mmax = 0;
  for (size_t q = 0; q < ps.size(); ++q) {
    BP& p = E.P[ps[q]];
    const OpSite& s = sites[q];
    eda_handle sb = p.sub;
    const bool use64 = master && sb->storage != EDA_F64;
    const char* base = use64 ? sb->P64.c() : sb->P.c();
    const char* Pc = base + (size_t)s.c0 * sb->ldp * dt_size(pdt);
    const double* sc = (pdt == DT::FP8) ? sb->pscale.d() + s.c0 : nullptr;
    v.push_back(TnArgs{p.d, s.Nc, s.nb, sb->ldp, s.ldv, 0, Pc, s.V, p.part, nullptr, sc});
    dmax = std::max(dmax, p.d);
    mmax = std::max(mmax, s.Nc);
  }
  for (auto& a : v) a.chunks = tn_chunks_for(a.d, dmax, mmax);
  std::vector<ReduceArgs> r;
  std::vector<NnArgs> core, out;
  for (size_t q = 0; q < ps.size(); ++q) {
    BP& p = E.P[ps[q]];
    const OpSite& s = sites[q];
    r.push_back(ReduceArgs{v[q].chunks, s.Nc, s.nb, 0, s.nb, p.part, 0.0, 0.0, 1.0, nullptr,
                           p.Ysm, nullptr});
    core.push_back(NnArgs{s.Nc, s.Nc, s.nb, s.ldc, s.nb, 0, s.nb, s.C, p.Ysm, 0.0, nullptr, p.Zsm,
                          1, nullptr});
    out.push_back(NnArgs{p.d, s.Nc, s.nb, p.sub->ldp, s.nb, s.ldv, s.ldo, v[q].A, p.Zsm, s.alpha,
                         s.V, s.Out, 0, nullptr, nullptr, v[q].ascale});
  }
  eda_handle h = E.h;
  hipStream_t st = h->stream;
  STCHK(push(h, std::move(v), [pdt, vdt, st](int cc, const TnArgs* hh, const TnArgs* dd) {
    return launch_tn_multi(cc, hh, dd, pdt, vdt, st);
  }));
  STCHK(push(h, std::move(r), [st](int cc, const ReduceArgs* hh, const ReduceArgs* dd) {
    return launch_reduce_multi(cc, hh, dd, st);
  }));
  STCHK(push(h, std::move(core), [st](int cc, const NnArgs* hh, const NnArgs* dd) {
    return launch_nn_multi(cc, hh, dd, DT::F64, DT::F64, DT::F64, st);
  }));
  STCHK(push(h, std::move(out), [pdt, vdt, odt, st](int cc, const NnArgs* hh, const NnArgs* dd) {
    return launch_nn_multi(cc, hh, dd, pdt, vdt, odt, st);
  }));
  return EDA_OK;
}

// ---- phases -------------------------------------------------------------------

eda_status lanczos_step(Engine& E, const std::vector<int>& ps, hipEvent_t e_op0,
                        hipEvent_t e_op1) {
  eda_handle h = E.h;
  const int64_t b = E.b;
  const DT qdt = E.qdt;
  const size_t qs = E.qs;
  STCHK(push_op(h, [h, e_op0]() { return hipEventRecord(e_op0, h->stream); }));
  // W goes straight into the slot of the next block, Q[:, m+b:m+2b]
  STCHK(m_expop(E, ps, qdt, qdt, [&](BP& p) {
    return OpSite{false, 0, p.N, p.sub->CM.d(), p.N, p.sub->alphaB, b, p.Qc(p.m, qs), p.ldq,
                  p.Qc(p.m + b, qs), p.ldq};
  }));
  STCHK(push_op(h, [h, e_op1]() { return hipEventRecord(e_op1, h->stream); }));
  STCHK(m_cgs(E, ps, qdt, [&](BP& p) {
    return CGSSite{p.Q[p.cur], p.ldq, p.m + b, p.Qc(p.m + b, qs), p.ldq, b,
                   p.H[p.cur] + p.m * p.ldh, p.ldh, 0.0, nullptr};
  }));
  // second pass and the Gram matrix of its result from one product:
  // [Q W]^T W = [h2; W^T W]; the Cholesky kernel forms W^T W - h2^T h2
  {
    int64_t dmax = 0, mmax = 0;
    for (int i : ps) {
      dmax = std::max(dmax, E.P[i].d);
      mmax = std::max(mmax, E.P[i].m + 2 * b);
    }
    STCHK(m_tn(E, ps, qdt, qdt, [&](BP& p) {
      return TnArgs{p.d, p.m + 2 * b, b, p.ldq, p.ldq, 0, p.Q[p.cur], p.Qc(p.m + b, qs), p.part,
                    nullptr};
    }));
    STCHK(m_reduce(E, ps, [&](BP& p) {
      ReduceArgs r{tn_chunks_for(p.d, dmax, mmax), p.m + 2 * b, b, p.ldh, b, p.part, 1.0, 1.0,
                   -1.0, p.H[p.cur] + p.m * p.ldh, p.hz, nullptr};
      r.mc = p.m + b;
      r.C2 = p.Gs;
      r.ldc2 = b;
      return r;
    }));
    STCHK(m_nn(E, ps, qdt, qdt, qdt, [&](BP& p) {
      return NnArgs{p.d, p.m + b, b, p.ldq, b, p.ldq, p.ldq, p.Q[p.cur], p.hz, 1.0,
                    p.Qc(p.m + b, qs), p.Qc(p.m + b, qs), 0, nullptr};
    }));
  }
  // rank-revealing first orthonormalisation (deflated directions replaced)
  STCHK(m_pchol(E, ps, [&](BP& p) {
    PcholArgs a{b, b, p.m + b, p.ldh, b, b, p.Gs, p.H[p.cur] + p.m * p.ldh, 1e-13, 1e-4, 0,
                p.Rinv, p.R1, p.mask, p.flags};
    a.corr = p.hz;
    a.mcorr = p.m + b;
    return a;
  }));
  STCHK(m_nn(E, ps, qdt, qdt, qdt, [&](BP& p) {
    return NnArgs{p.d, b, b, p.ldq, b, p.ldq, p.ldq, p.Qc(p.m + b, qs), p.Rinv, 0.0, nullptr,
                  p.Qc(p.m + b, qs), 0, nullptr};
  }));
  STCHK(m_mrandn(E, ps, qdt, [&](BP& p) {
    return MaskedRandnArgs{p.d, b, p.ldq, p.mask, 0x5eed0000ull + (uint64_t)p.m,
                           p.Qc(p.m + b, qs)};
  }));
  STCHK(m_cholqr(E, ps, qdt, [&](BP& p) {
    return QRSite{p.Qc(p.m + b, qs), p.ldq, p.Qc(p.m + b, qs), p.ldq, b, p.R1,
                  p.H[p.cur] + (p.m + b) + p.m * p.ldh, p.ldh, p.flags, nullptr};
  }));
  // repair, gated on the flag raised above
  for (int pass = 0; pass < 2; ++pass)
    STCHK(m_cgs(E, ps, qdt, [&](BP& p) {
      return CGSSite{p.Q[p.cur], p.ldq, p.m + b, p.Qc(p.m + b, qs), p.ldq, b, nullptr, 0, 0.0,
                     p.flags};
    }));
  for (int pass = 0; pass < 2; ++pass)
    STCHK(m_cholqr(E, ps, qdt, [&](BP& p) {
      return QRSite{p.Qc(p.m + b, qs), p.ldq, p.Qc(p.m + b, qs), p.ldq, b, nullptr, nullptr, 0,
                    p.flags, p.flags};
    }));
  STCHK(m_fold(E, ps, [&](BP& p) { return FlagArgs{p.flags}; }));
  return EDA_OK;
}

// Rayleigh-Ritz on Q[:, 0:m] for each listed problem with its own count of
// wanted values; theta/est land in the pinned readback slots.
eda_status rayleigh_ritz(Engine& E, const std::vector<int>& ps, const std::vector<int64_t>& cnt) {
  eda_handle h = E.h;
  const int64_t b = E.b;
  STCHK(m_sym(E, ps, [&](BP& p) { return SymArgs{p.m, p.ldh, p.mmax, p.H[p.cur], p.T}; }));
  STCHK(m_syev(E, ps, [&](BP& p) {
    return SyevArgs{p.m, p.mmax, p.mmax, std::min<int64_t>(std::min<int64_t>(p.kk, p.mmax), p.m),
                    p.T, p.wT, p.S, p.syw};
  }));
  size_t q = 0;
  std::vector<int64_t> cc(cnt);
  STCHK(m_ritzest(E, ps, [&](BP& p) {
    const int64_t c = cc[q++];
    return RitzEstArgs{p.m, b, c, p.mmax, p.ldh, p.wT, p.S, p.H[p.cur] + p.m + (p.m - b) * p.ldh,
                       p.dtheta, p.dres};
  }));
  for (size_t i = 0; i < ps.size(); ++i) {
    BP* p = &E.P[ps[i]];
    const int64_t c = cnt[i];
    STCHK(push_op(h, [h, p, c]() {
      hipError_t e = hipMemcpyAsync(p->hth, p->dtheta, c * 8, hipMemcpyDeviceToHost, h->stream);
      if (e != hipSuccess) return e;
      e = hipMemcpyAsync(p->hre, p->dres, c * 8, hipMemcpyDeviceToHost, h->stream);
      if (e != hipSuccess) return e;
      return hipMemcpyAsync(p->hfl, p->flags, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream);
    }));
  }
  STCHK(stage_run(h));
  HIPCHK(hipStreamSynchronize(h->stream));
  for (size_t i = 0; i < ps.size(); ++i) {
    BP& p = E.P[ps[i]];
    p.theta.assign(p.hth, p.hth + cnt[i]);
    p.est.assign(p.hre, p.hre + cnt[i]);
    p.m_rr = p.m;
  }
  return EDA_OK;
}

eda_status thick_restart(Engine& E, const std::vector<int>& ps) {
  const int64_t b = E.b;
  const DT qdt = E.qdt;
  const size_t qs = E.qs;
  STCHK(m_gather(E, ps, [&](BP& p) { return GatherArgs{p.m, p.kk, p.mmax, p.kk, p.S, p.Sd}; }));
  STCHK(m_nn(E, ps, qdt, qdt, qdt, [&](BP& p) {
    return NnArgs{p.d, p.m, p.kk, p.ldq, p.kk, p.ldq, p.ldq, p.Q[p.cur], p.Sd, 0.0, nullptr,
                  p.Q[1 - p.cur], 0, nullptr};
  }));
  STCHK(m_copy(E, ps, qdt, qdt, [&](BP& p) {
    return Copy2dArgs{p.d, b, p.ldq, p.ldq, p.Qc(p.m, qs), p.Q[1 - p.cur] + (size_t)p.kk * p.ldq * qs};
  }));
  STCHK(m_fill(E, ps, [&](BP& p) { return FillArgs{p.ldh * p.ldh, 0.0, p.H[1 - p.cur]}; }));
  STCHK(m_setdiag(E, ps, [&](BP& p) { return SetDiagArgs{p.kk, p.ldh, p.dtheta, p.H[1 - p.cur]}; }));
  STCHK(m_coupling(E, ps, [&](BP& p) {
    return CouplingArgs{p.m, b, p.kk, p.ldh, p.kk, p.ldh, p.H[p.cur] + p.m + (p.m - b) * p.ldh,
                        p.Sd, p.H[1 - p.cur]};
  }));
  for (int i : ps) {
    BP& p = E.P[i];
    p.cur = 1 - p.cur;
    p.m = p.kk;
    ++p.restarts;
  }
  return EDA_OK;
}

// Float64 Rayleigh-Ritz on the w columns of XB[cb] (MB[cb] = M of them):
// top t to XB[1-cb], MB[1-cb], Ritz values to dtheta.
eda_status rr_block(Engine& E, const std::vector<int>& ps, const std::vector<int64_t>& ws) {
  size_t q;
  q = 0;
  STCHK(m_tn(E, ps, DT::F64, DT::F64, [&](BP& p) {
    const int64_t w = ws[q++];
    return TnArgs{p.d, w, w, p.ldq, p.ldq, 0, p.XB[p.cb], p.MB[p.cb], p.part, nullptr};
  }));
  {
    int64_t dmax = 0, wmax = 0;
    for (size_t i = 0; i < ps.size(); ++i) {
      dmax = std::max(dmax, E.P[ps[i]].d);
      wmax = std::max(wmax, ws[i]);
    }
    q = 0;
    STCHK(m_reduce(E, ps, [&](BP& p) {
      const int64_t w = ws[q++];
      return ReduceArgs{tn_chunks_for(p.d, dmax, wmax), w, w, p.mm, 0, p.part, 1.0, 0.0, 0.0, p.S,
                        nullptr, nullptr};
    }));
  }
  q = 0;
  STCHK(m_sym(E, ps, [&](BP& p) { return SymArgs{ws[q++], p.mm, p.mm, p.S, p.T}; }));
  q = 0;
  STCHK(m_syev(E, ps, [&](BP& p) {
    return SyevArgs{ws[q++], p.mm, p.mm, p.t, p.T, p.wT, p.S, p.syw};
  }));
  q = 0;
  STCHK(m_gather(E, ps, [&](BP& p) { return GatherArgs{ws[q++], p.t, p.mm, p.t, p.S, p.Sd}; }));
  q = 0;
  STCHK(m_desc(E, ps, [&](BP& p) { return DescArgs{p.t, ws[q++], p.wT, p.dtheta}; }));
  q = 0;
  STCHK(m_nn(E, ps, DT::F64, DT::F64, DT::F64, [&](BP& p) {
    return NnArgs{p.d, ws[q++], p.t, p.ldq, p.t, p.ldq, p.ldq, p.XB[p.cb], p.Sd, 0.0, nullptr,
                  p.XB[1 - p.cb], 0, nullptr};
  }));
  q = 0;
  STCHK(m_nn(E, ps, DT::F64, DT::F64, DT::F64, [&](BP& p) {
    return NnArgs{p.d, ws[q++], p.t, p.ldq, p.t, p.ldq, p.ldq, p.MB[p.cb], p.Sd, 0.0, nullptr,
                  p.MB[1 - p.cb], 0, nullptr};
  }));
  for (int i : ps) E.P[i].cb = 1 - E.P[i].cb;
  return EDA_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

extern "C" eda_status eda_solve_batched(eda_handle h, int32_t count, const eda_problem* probs,
                                        eda_dtype storage, const eda_solve_opts* opt,
                                        eda_info* infos, eda_status* statuses) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (count < 1 || count > 4096) return fail(h, EDA_ERR_ARG, "count must be in [1, 4096]");
  if (probs == nullptr) return fail(h, EDA_ERR_ARG, "null problem array");
  eda_solve_opts o;
  std::memset(&o, 0, sizeof(o));
  if (opt != nullptr) o = *opt;
  if (o.form != EDA_FORM_LANCZOS_M) return fail(h, EDA_ERR_ARG, "only the Lanczos form is solved");
  if (o.krylov_dtype != EDA_F64 && o.krylov_dtype != EDA_F32)
    return fail(h, EDA_ERR_ARG, "krylov_dtype (basis type) must be EDA_F64 or EDA_F32");
  if (o.refine_dtype != EDA_F64) return fail(h, EDA_ERR_ARG, "refine_dtype must be EDA_F64");
  if (o.resmode != EDA_RES_REL_THETA && o.resmode != EDA_RES_NORMWISE)
    return fail(h, EDA_ERR_ARG, "unknown residual mode");
  if (o.start_block != nullptr) return fail(h, EDA_ERR_ARG, "start_block is not used in batches");
  if (storage != EDA_F64 && storage != EDA_F32 && storage != EDA_BF16 && storage != EDA_FP8_E4M3)
    return fail(h, EDA_ERR_ARG, "storage must be EDA_F64, EDA_F32, EDA_BF16 or EDA_FP8_E4M3");
  const int64_t b = o.block > 0 ? o.block : 8;
  if (b > 8) return fail(h, EDA_ERR_ARG, "block width must be in [1, 8]");
  if (o.max_basis > 0) return fail(h, EDA_ERR_ARG, "max_basis is chosen per problem in batches");
  for (int32_t p = 0; p < count; ++p) {
    const eda_problem& q = probs[p];
    if (q.d < 2 || q.k < 2 || q.n < q.k || q.n + q.k > 2048)
      return fail(h, EDA_ERR_ARG, "problem %d: need d>=2, 2<=k<=n, n+k<=2048", (int)p);
    if (q.H_W == nullptr || q.H_B == nullptr || q.X == nullptr || q.ritz == nullptr ||
        q.ritz_log == nullptr || q.resid == nullptr)
      return fail(h, EDA_ERR_ARG, "problem %d: null pointer", (int)p);
    if (q.ldw < q.d || q.ldb < q.d || q.ldx < q.d)
      return fail(h, EDA_ERR_ARG, "problem %d: leading dimensions must be >= d", (int)p);
    if (q.t < 1 || q.t >= q.d || q.t > 128)
      return fail(h, EDA_ERR_ARG, "problem %d: need 1 <= t <= 128, t < d", (int)p);
    if (!(q.tol > 0.0) || !std::isfinite(q.tol))
      return fail(h, EDA_ERR_ARG, "problem %d: tol must be positive", (int)p);
    const int64_t mmax0 = std::min<int64_t>(
        std::min<int64_t>(round_up(std::max<int64_t>(2 * q.t + 2 * b, q.t + 6 * b), b), q.d),
        2048 - b);
    if (mmax0 < q.t + 2 * b)
      return fail(h, EDA_ERR_ARG, "problem %d: d too small for t and the block", (int)p);
  }
  STCHK(need_device(h));
  for (int32_t p = 0; p < count; ++p) STCHK(check_dev_ptr(h, probs[p].X, "X"));
  {
    // launch shapes of the product passes, measured once per shape class of
    // the largest problem (EDA_AUTOTUNE=0 keeps the size heuristics)
    int64_t dmax = 0, Nmax = 0;
    for (int32_t p = 0; p < count; ++p) {
      dmax = std::max<int64_t>(dmax, probs[p].d);
      Nmax = std::max<int64_t>(Nmax, probs[p].n + probs[p].k);
    }
    const char* at = std::getenv("EDA_AUTOTUNE");
    const bool tune = at == nullptr || std::strcmp(at, "0") != 0;
    if (tune && tune_get(TuneKind::TnSteps, dmax, Nmax, 0) < 0)
      STCHK(autotune_shapes(h, dmax, Nmax, b, storage, nullptr, nullptr, nullptr));
  }

  if (h->batch == nullptr) h->batch = new BatchState();
  BatchState* Bs = h->batch;
  ArgStage& st = Bs->st;
  if (st.dev == nullptr) {
    for (int q = 0; q < 2; ++q) {
      if (hipHostMalloc((void**)&st.host[q], kStageBytes, hipHostMallocDefault) != hipSuccess)
        return fail(h, EDA_ERR_NOMEM, "pinned staging allocation failed");
      HIPCHK(hipEventCreate(&st.ev[q]));
    }
    if (hipMalloc((void**)&st.dev, kStageBytes) != hipSuccess)
      return fail(h, EDA_ERR_NOMEM, "device staging allocation failed");
    st.cap = kStageBytes;
  }
  while ((int32_t)Bs->subs.size() < count) {
    eda_handle sb = nullptr;
    const eda_status s0 = eda_create(&sb, (void*)h->stream);
    if (s0 != EDA_OK) {
      if (sb != nullptr) eda_destroy(sb);
      return fail(h, s0, "internal handle creation failed");
    }
    sb->poly_readback = false;
    Bs->subs.push_back(sb);
  }
  while (Bs->ev.size() < 4) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    Bs->ev.push_back(e);
  }
  hipStream_t s = h->stream;
  hipEvent_t ev_t0 = Bs->ev[0], ev_t1 = Bs->ev[1], ev_t2 = Bs->ev[2];
  HIPCHK(hipEventRecord(ev_t0, s));

  // ---- a1-a3 for every problem: one drain of the stream in the middle -------
  std::vector<eda_status> stat(count, EDA_OK);
  for (int32_t p = 0; p < count; ++p) {
    const eda_problem& q = probs[p];
    stat[p] = prepare_begin(Bs->subs[p], q.d, q.n, q.k, q.H_W, q.ldw, q.H_B, q.ldb, storage);
    if (stat[p] != EDA_OK) return fail(h, stat[p], "problem %d: %s", (int)p, Bs->subs[p]->err.c_str());
  }
  HIPCHK(hipStreamSynchronize(s));
  for (int32_t p = 0; p < count; ++p) {
    stat[p] = prepare_end(Bs->subs[p]);
    if (stat[p] != EDA_OK) return fail(h, stat[p], "problem %d: %s", (int)p, Bs->subs[p]->err.c_str());
  }
  HIPCHK(hipEventRecord(ev_t1, s));

  // ---- engine set-up ---------------------------------------------------------
  Engine E;
  E.h = h;
  E.b = b;
  E.qdt = o.krylov_dtype == EDA_F32 ? DT::F32 : DT::F64;
  E.sdt = dt_of(storage);
  E.qs = dt_size(E.qdt);
  E.mixed = (storage != EDA_F64) || (E.qdt != DT::F64);
  E.u_lo = std::max(unit_roundoff(E.sdt), unit_roundoff(E.qdt));
  E.check_every = o.check_every > 0 ? o.check_every : 2;
  E.max_iter = o.max_iter > 0 ? o.max_iter : 4000;
  E.max_refine = o.max_refine > 0 ? o.max_refine : (o.max_refine < 0 ? -1 : (E.mixed ? 16 : 2));
  E.resmode = o.resmode;
  E.seed = o.seed;
  E.P.resize(count);
  size_t total = 0;
  std::vector<size_t> sizes;
  int64_t mm_all = 0;
  for (int32_t p = 0; p < count; ++p) {
    BP& P = E.P[p];
    const eda_problem& q = probs[p];
    P.sub = Bs->subs[p];
    P.pr = &q;
    P.t = q.t;
    P.tol = q.tol;
    P.d = q.d;
    P.n = q.n;
    P.k = q.k;
    P.N = q.n + q.k;
    P.ldq = P.sub->ldp;
    P.mmax = std::min<int64_t>(
        std::min<int64_t>(round_up(std::max<int64_t>(2 * P.t + 2 * b, P.t + 6 * b), b), P.d),
        2048 - b);
    P.ldh = P.mmax + b;
    P.kk = std::max<int64_t>(P.t, std::min<int64_t>(P.t + b, P.mmax - 2 * b));
    P.wz = std::min<int64_t>(P.t, P.d - P.t);
    P.mm = std::max<int64_t>(P.mmax, P.t + P.wz);
    P.bt = std::max<int64_t>(b, P.t);
    mm_all = std::max(mm_all, P.mm);
  }
  E.mm_all = mm_all;
  // per-problem workspace, one arena
  struct Slot { size_t off, bytes; };
  std::vector<std::vector<Slot>> slots(count);
  for (int32_t p = 0; p < count; ++p) {
    BP& P = E.P[p];
    const int64_t t = P.t, wz = P.wz, bt = P.bt;
    const int64_t rb = std::max<int64_t>(b, std::min<int64_t>(wz, 64));
    const int64_t shapes[][2] = {{P.N, b},   {P.mmax + b, b}, {b, b},  {P.N, t},        {P.n, t},
                                 {t, t},     {t, wz},         {wz, wz}, {t + wz, t + wz}, {P.mmax, P.kk}};
    int64_t mn = 0;
    for (const auto& sh : shapes) mn = std::max(mn, sh[0] * sh[1]);
    const size_t part_b = (size_t)((P.d + 255) / 256) * mn * 8;
    const size_t bytes[] = {
        (size_t)P.ldq * (P.mmax + b) * E.qs, (size_t)P.ldq * (P.mmax + b) * E.qs,  // Q[2]
        (size_t)P.ldh * P.ldh * 8, (size_t)P.ldh * P.ldh * 8,                      // H[2]
        (size_t)P.ldq * b * E.qs,                                                  // W
        (size_t)P.ldq * std::max<int64_t>(t, b) * 8,                               // Yb
        (size_t)P.mm * P.mm * 8, (size_t)P.mm * P.mm * 8, (size_t)P.mm * 8,        // T S wT
        (size_t)std::max(P.mmax * P.kk, (t + wz) * t) * 8,                         // Sd
        part_b,                                                                    // part
        (size_t)P.N * bt * 8, (size_t)P.N * bt * 8,                                // Ysm Zsm
        (size_t)std::max<int64_t>((P.mmax + b) * b, t * t) * 8,                    // hz
        (size_t)bt * bt * 8, (size_t)bt * bt * 8, (size_t)rb * rb * 8,             // Gs Rinv R1
        (size_t)(P.kk + 8) * 8, (size_t)(P.kk + 8) * 8,                            // dtheta dres
        syev_work_bytes(mm_all),                                                   // syev work
        (size_t)8 * P.ldq * t * 8,                                                 // refine
        64, 128 * sizeof(int)};                                                    // flags mask
    for (size_t by : bytes) {
      slots[p].push_back(Slot{total, by});
      total += align256(by);
    }
  }
  if (Bs->arena_cap < total) {
    if (Bs->arena != nullptr) {
      HIPCHK(hipStreamSynchronize(s));
      (void)hipFree(Bs->arena);
      Bs->arena = nullptr;
      Bs->arena_cap = 0;
    }
    if (hipMalloc(&Bs->arena, total) != hipSuccess) {
      (void)hipGetLastError();
      return fail(h, EDA_ERR_NOMEM, "batch workspace of %zu bytes failed", total);
    }
    Bs->arena_cap = total;
  }
  int64_t kmax = 0;
  for (auto& P : E.P) kmax = std::max(kmax, P.kk + 8);
  const size_t hp_bytes = (size_t)count * (2 * kmax + 2) * 8;
  if (Bs->hpin_cap < hp_bytes) {
    if (Bs->hpin != nullptr) (void)hipHostFree(Bs->hpin);
    Bs->hpin = nullptr;
    if (hipHostMalloc((void**)&Bs->hpin, hp_bytes, hipHostMallocDefault) != hipSuccess)
      return fail(h, EDA_ERR_NOMEM, "pinned readback allocation failed");
    Bs->hpin_cap = hp_bytes;
  }
  char* ar = (char*)Bs->arena;
  for (int32_t p = 0; p < count; ++p) {
    BP& P = E.P[p];
    auto at = [&](int i) { return ar + slots[p][i].off; };
    P.Q[0] = at(0);
    P.Q[1] = at(1);
    P.H[0] = (double*)at(2);
    P.H[1] = (double*)at(3);
    P.W = at(4);
    P.Yb = (double*)at(5);
    P.T = (double*)at(6);
    P.S = (double*)at(7);
    P.wT = (double*)at(8);
    P.Sd = (double*)at(9);
    P.part = (double*)at(10);
    P.Ysm = (double*)at(11);
    P.Zsm = (double*)at(12);
    P.hz = (double*)at(13);
    P.Gs = (double*)at(14);
    P.Rinv = (double*)at(15);
    P.R1 = (double*)at(16);
    P.dtheta = (double*)at(17);
    P.dres = (double*)at(18);
    P.syw = (double*)at(19);
    P.refine = (double*)at(20);
    P.flags = (int*)at(21);
    P.mask = (int*)at(22);
    const size_t rw = (size_t)P.ldq * 2 * P.t;
    P.XB[0] = P.refine;
    P.XB[1] = P.refine + rw;
    P.MB[0] = P.refine + 2 * rw;
    P.MB[1] = P.refine + 3 * rw;
    P.hth = Bs->hpin + (size_t)p * (2 * kmax + 2);
    P.hre = P.hth + kmax;
    P.hfl = (int*)(P.hre + kmax);
    if (P.t > P.k - 1) P.flags_out |= EDA_WARN_DEGENERATE;
  }

  std::vector<int> all(count);
  for (int32_t p = 0; p < count; ++p) all[p] = p;
  const DT qdt = E.qdt;
  const size_t qs = E.qs;

  // ---- start blocks ------------------------------------------------------------
  STCHK(m_fill_i32(E, all, [&](BP& p) { return FillI32Args{16, 0, p.flags}; }));
  for (int q = 0; q < 2; ++q)
    STCHK(m_fill(E, all, [&](BP& p) { return FillArgs{p.ldh * p.ldh, 0.0, p.H[q]}; }));
  {
    int32_t pi = 0;
    STCHK(m_randn(E, all, [&](BP& p) {
      return RandnArgs{p.d, b, p.ldq, o.seed + (uint64_t)(pi++), p.Yb};
    }));
  }
  STCHK(m_copy(E, all, DT::F64, qdt, [&](BP& p) {
    return Copy2dArgs{p.d, b, p.ldq, p.ldq, p.Yb, p.W};
  }));
  if (qdt == DT::F64)
    STCHK(m_fill(E, all, [&](BP& p) {
      return FillArgs{p.ldq * (p.mmax + b), 0.0, (double*)p.Q[0]};
    }));
  else  // float32 zero has the bit pattern of int32 zero
    STCHK(m_fill_i32(E, all, [&](BP& p) {
      return FillI32Args{p.ldq * (p.mmax + b), 0, (int*)p.Q[0]};
    }));
  STCHK(m_cholqr(E, all, qdt, [&](BP& p) {
    return QRSite{p.W, p.ldq, p.Q[0], p.ldq, b, nullptr, nullptr, 0, nullptr, nullptr};
  }));
  STCHK(m_cholqr(E, all, qdt, [&](BP& p) {
    return QRSite{p.Q[0], p.ldq, p.Q[0], p.ldq, b, nullptr, nullptr, 0, nullptr, nullptr};
  }));

  // ---- Krylov phase, all problems in lockstep ----------------------------------
  std::vector<hipEvent_t> opev;
  int64_t step = 0;
  std::vector<std::vector<int>> step_members;
  while (true) {
    std::vector<int> act;
    for (int32_t p = 0; p < count; ++p)
      if (E.P[p].active) act.push_back(p);
    if (act.empty()) break;
    if (opev.size() < (size_t)(2 * step + 2)) {
      for (int q = 0; q < 2; ++q) {
        hipEvent_t e;
        HIPCHK(hipEventCreate(&e));
        opev.push_back(e);
      }
    }
    STCHK(lanczos_step(E, act, opev[2 * step], opev[2 * step + 1]));
    step_members.push_back(act);
    ++step;
    std::vector<int> chk, fin;
    std::vector<int64_t> cnt;
    for (int p : act) {
      BP& P = E.P[p];
      P.m += b;
      ++P.iters;
      P.ops += b;
      P.bytes += 2.0 * P.d * P.N * dsize(storage) + 3.0 * P.d * b * qs;
      ++P.op_calls;
      const bool need_restart = (P.m + b > P.mmax);
      const bool can_check = (P.m >= P.t + b) || need_restart;
      if (can_check && (P.iters % E.check_every == 0 || need_restart || P.iters >= E.max_iter)) {
        chk.push_back(p);
        cnt.push_back(need_restart ? P.kk : P.t);
      } else if (P.iters >= E.max_iter) {
        chk.push_back(p);
        cnt.push_back(std::min<int64_t>(P.t, P.m));
        fin.push_back(p);
      }
    }
    if (chk.empty()) {
      STCHK(stage_run(h));
      continue;
    }
    STCHK(rayleigh_ritz(E, chk, cnt));
    std::vector<int> rs;
    for (int p : chk) {
      BP& P = E.P[p];
      if (std::find(fin.begin(), fin.end(), p) != fin.end()) {
        P.active = false;
        continue;
      }
      bool ok = true;
      const double th1 = P.theta[0];
      for (int64_t i = 0; i < P.t; ++i) {
        const double thi = P.theta[i];
        if (!(thi > 0.0)) { ok = false; continue; }
        const double tol_i = std::max(P.tol, 10.0 * E.u_lo * th1 / thi);
        const double r = (E.resmode == EDA_RES_REL_THETA) ? P.est[i] / thi : P.est[i] / th1;
        if (!(r <= tol_i)) ok = false;
      }
      if (ok) {
        P.kconv = true;
        P.active = false;
      } else if (P.iters >= E.max_iter) {
        P.active = false;
      } else if (P.m + b > P.mmax) {
        rs.push_back(p);
      }
    }
    if (!rs.empty()) STCHK(thick_restart(E, rs));
  }
  // final Rayleigh-Ritz where the last one is stale
  {
    std::vector<int> ps;
    std::vector<int64_t> cnt;
    for (int32_t p = 0; p < count; ++p) {
      BP& P = E.P[p];
      if (P.m < P.t) {
        stat[p] = EDA_ERR_NOCONV;
        continue;
      }
      if (P.m_rr != P.m) {
        ps.push_back(p);
        cnt.push_back(P.t);
      }
    }
    if (!ps.empty()) STCHK(rayleigh_ritz(E, ps, cnt));
  }
  std::vector<int> live;
  for (int32_t p = 0; p < count; ++p)
    if (stat[p] == EDA_OK) live.push_back(p);

  // Ritz vectors Y = Q S_t in float64
  STCHK(m_gather(E, live, [&](BP& p) { return GatherArgs{p.m, p.t, p.mmax, p.t, p.S, p.Sd}; }));
  STCHK(m_nn(E, live, qdt, DT::F64, DT::F64, [&](BP& p) {
    return NnArgs{p.d, p.m, p.t, p.ldq, p.t, p.ldq, p.ldq, p.Q[p.cur], p.Sd, 0.0, nullptr,
                  p.XB[0], 0, nullptr};
  }));
  STCHK(push_op(h, [h, ev_t2]() { return hipEventRecord(ev_t2, h->stream); }));

  // ---- float64 stage -------------------------------------------------------------
  auto op64 = [&](const std::vector<int>& ps, bool expansion) {
    return m_expop(E, ps, DT::F64, DT::F64, [&](BP& p) {
      const int64_t cols = expansion ? p.wz : p.t;
      const double* V = expansion ? p.XB[p.cb] + (size_t)p.t * p.ldq : p.XB[p.cb];
      double* Out = expansion ? p.MB[p.cb] + (size_t)p.t * p.ldq : p.MB[p.cb];
      return OpSite{true, 0, p.N, p.sub->CM.d(), p.N, p.sub->alphaB, cols, V, p.ldq, Out, p.ldq};
    });
  };
  if (E.mixed && E.max_refine >= 0) {
    STCHK(m_cholqr(E, live, DT::F64, [&](BP& p) {
      return QRSite{p.XB[0], p.ldq, p.Yb, p.ldq, p.t, nullptr, nullptr, 0, nullptr, nullptr};
    }));
    STCHK(m_cholqr(E, live, DT::F64, [&](BP& p) {
      return QRSite{p.Yb, p.ldq, p.XB[0], p.ldq, p.t, nullptr, nullptr, 0, nullptr, nullptr};
    }));
    STCHK(op64(live, false));
    std::vector<int64_t> ws;
    for (int p : live) {
      E.P[p].ops += E.P[p].t;
      E.P[p].bytes += 2.0 * E.P[p].d * E.P[p].N * 8.0 + 3.0 * E.P[p].d * E.P[p].t * 8.0;
      ws.push_back(E.P[p].t);
    }
    STCHK(rr_block(E, live, ws));
  } else {
    STCHK(op64(live, false));
    for (int p : live) {
      E.P[p].ops += E.P[p].t;
      E.P[p].bytes += 2.0 * E.P[p].d * E.P[p].N * 8.0 + 3.0 * E.P[p].d * E.P[p].t * 8.0;
    }
  }
  std::vector<int> ref(live);
  while (!ref.empty()) {
    STCHK(m_resid(E, ref, [&](BP& p) {
      return ResidArgs{p.d, p.t, p.ldq, p.ldq, p.ldq, p.MB[p.cb], p.XB[p.cb], p.dtheta,
                       p.XB[p.cb] + (size_t)p.t * p.ldq, p.dres};
    }));
    for (int pi : ref) {
      BP* p = &E.P[pi];
      STCHK(push_op(h, [h, p]() {
        hipError_t e = hipMemcpyAsync(p->hth, p->dtheta, p->t * 8, hipMemcpyDeviceToHost, h->stream);
        if (e != hipSuccess) return e;
        return hipMemcpyAsync(p->hre, p->dres, p->t * 8, hipMemcpyDeviceToHost, h->stream);
      }));
    }
    STCHK(stage_run(h));
    HIPCHK(hipStreamSynchronize(s));
    std::vector<int> more;
    for (int pi : ref) {
      BP& P = E.P[pi];
      P.theta.assign(P.hth, P.hth + P.t);
      P.est.assign(P.hre, P.hre + P.t);
      bool ok = true;
      P.floor_limited = false;
      const double th1 = P.theta[0];
      for (int64_t i = 0; i < P.t; ++i) {
        const double thi = P.theta[i];
        if (!(thi > 0.0)) { ok = false; continue; }
        const double floor_i = 10.0 * kU64 * th1 / thi;
        if (floor_i > P.tol) P.floor_limited = true;
        const double r = (E.resmode == EDA_RES_REL_THETA) ? P.est[i] / thi : P.est[i] / th1;
        if (!(r <= std::max(P.tol, floor_i))) ok = false;
      }
      if (ok) {
        P.converged = true;
      } else if (P.kconv && P.passes < E.max_refine) {
        more.push_back(pi);
      }
    }
    if (more.empty()) break;
    // expansion by the orthonormalised residual block (2t > d keeps the last wz)
    {
      std::vector<int> shr;
      for (int pi : more)
        if (E.P[pi].wz < E.P[pi].t) shr.push_back(pi);
      STCHK(m_copy(E, shr, DT::F64, DT::F64, [&](BP& p) {
        return Copy2dArgs{p.d, p.wz, p.ldq, p.ldq, p.XB[p.cb] + (size_t)(2 * p.t - p.wz) * p.ldq,
                          p.Yb};
      }));
      STCHK(m_copy(E, shr, DT::F64, DT::F64, [&](BP& p) {
        return Copy2dArgs{p.d, p.wz, p.ldq, p.ldq, p.Yb, p.XB[p.cb] + (size_t)p.t * p.ldq};
      }));
    }
    auto Zp = [](BP& p) { return p.XB[p.cb] + (size_t)p.t * p.ldq; };
    for (int pass = 0; pass < 2; ++pass)
      STCHK(m_cgs(E, more, DT::F64, [&](BP& p) {
        return CGSSite{p.XB[p.cb], p.ldq, p.t, Zp(p), p.ldq, p.wz, nullptr, 0, 0.0, nullptr};
      }));
    std::vector<int> small, wide;
    for (int pi : more) (E.P[pi].wz <= 64 ? small : wide).push_back(pi);
    if (!small.empty()) {
      STCHK(m_tn(E, small, DT::F64, DT::F64, [&](BP& p) {
        return TnArgs{p.d, p.wz, p.wz, p.ldq, p.ldq, 0, Zp(p), Zp(p), p.part, nullptr};
      }));
      int64_t dmax = 0, wmax = 0;
      for (int pi : small) {
        dmax = std::max(dmax, E.P[pi].d);
        wmax = std::max(wmax, E.P[pi].wz);
      }
      STCHK(m_reduce(E, small, [&](BP& p) {
        return ReduceArgs{tn_chunks_for(p.d, dmax, wmax), p.wz, p.wz, p.wz, 0, p.part, 1.0, 0.0,
                          0.0, p.Gs, nullptr, nullptr};
      }));
      STCHK(m_pchol(E, small, [&](BP& p) {
        return PcholArgs{p.wz, p.wz, 0, 0, p.wz, p.wz, p.Gs, nullptr, 1e-10, 1e-4, 1, p.Rinv, p.R1,
                         p.mask, nullptr};
      }));
      STCHK(m_nn(E, small, DT::F64, DT::F64, DT::F64, [&](BP& p) {
        return NnArgs{p.d, p.wz, p.wz, p.ldq, p.wz, p.ldq, p.ldq, Zp(p), p.Rinv, 0.0, nullptr,
                      p.Yb, 0, nullptr};
      }));
      STCHK(m_mrandn(E, small, DT::F64, [&](BP& p) {
        return MaskedRandnArgs{p.d, p.wz, p.ldq, p.mask, 0x7e41e000ull + (uint64_t)p.passes, p.Yb};
      }));
      for (int pass = 0; pass < 2; ++pass)
        STCHK(m_cgs(E, small, DT::F64, [&](BP& p) {
          return CGSSite{p.XB[p.cb], p.ldq, p.t, p.Yb, p.ldq, p.wz, nullptr, 0, 0.0, nullptr};
        }));
      STCHK(m_cholqr(E, small, DT::F64, [&](BP& p) {
        return QRSite{p.Yb, p.ldq, Zp(p), p.ldq, p.wz, nullptr, nullptr, 0, nullptr, nullptr};
      }));
    }
    if (!wide.empty()) {
      STCHK(m_cholqr(E, wide, DT::F64, [&](BP& p) {
        return QRSite{Zp(p), p.ldq, p.Yb, p.ldq, p.wz, nullptr, nullptr, 0, nullptr, nullptr};
      }));
      STCHK(m_cgs(E, wide, DT::F64, [&](BP& p) {
        return CGSSite{p.XB[p.cb], p.ldq, p.t, p.Yb, p.ldq, p.wz, nullptr, 0, 0.0, nullptr};
      }));
      STCHK(m_cholqr(E, wide, DT::F64, [&](BP& p) {
        return QRSite{p.Yb, p.ldq, Zp(p), p.ldq, p.wz, nullptr, nullptr, 0, nullptr, nullptr};
      }));
    }
    STCHK(m_cholqr(E, more, DT::F64, [&](BP& p) {
      return QRSite{Zp(p), p.ldq, p.Yb, p.ldq, p.wz, nullptr, nullptr, 0, nullptr, nullptr};
    }));
    STCHK(m_copy(E, more, DT::F64, DT::F64, [&](BP& p) {
      return Copy2dArgs{p.d, p.wz, p.ldq, p.ldq, p.Yb, Zp(p)};
    }));
    STCHK(op64(more, true));
    std::vector<int64_t> ws;
    for (int pi : more) {
      BP& P = E.P[pi];
      P.ops += P.wz;
      P.bytes += 2.0 * P.d * P.N * 8.0 + 3.0 * P.d * P.wz * 8.0;
      ws.push_back(P.t + P.wz);
      ++P.passes;
    }
    STCHK(rr_block(E, more, ws));
    ref = more;
  }
  STCHK(push_op(h, [h, Bs]() { return hipEventRecord(Bs->ev[3], h->stream); }));

  // back-transform x = exp(-S_W/2) y, orthonormalise (Cholesky QR twice), signs
  STCHK(m_expop(E, live, DT::F64, DT::F64, [&](BP& p) {
    return OpSite{true, 0, p.n, p.sub->Gh.d(), p.n, 1.0, p.t, p.XB[p.cb], p.ldq, p.pr->X,
                  p.pr->ldx};
  }));
  STCHK(m_cholqr(E, live, DT::F64, [&](BP& p) {
    return QRSite{p.pr->X, p.pr->ldx, p.Yb, p.ldq, p.t, nullptr, nullptr, 0, nullptr, nullptr};
  }));
  STCHK(m_cholqr(E, live, DT::F64, [&](BP& p) {
    return QRSite{p.Yb, p.ldq, p.pr->X, p.pr->ldx, p.t, nullptr, nullptr, 0, nullptr, nullptr};
  }));
  STCHK(m_sign(E, live, [&](BP& p) { return SignArgs{p.d, p.t, p.pr->ldx, p.pr->X}; }));
  for (int pi : live) {
    BP* p = &E.P[pi];
    STCHK(push_op(h, [h, p]() {
      return hipMemcpyAsync(p->hfl, p->flags, 2 * sizeof(int), hipMemcpyDeviceToHost, h->stream);
    }));
  }
  STCHK(stage_run(h));
  HIPCHK(hipStreamSynchronize(s));

  float prep_ms = 0.f, kry_ms = 0.f, ref_ms = 0.f;
  HIPCHK(hipEventElapsedTime(&prep_ms, ev_t0, ev_t1));
  HIPCHK(hipEventElapsedTime(&kry_ms, ev_t1, ev_t2));
  HIPCHK(hipEventElapsedTime(&ref_ms, ev_t2, Bs->ev[3]));
  std::vector<double> step_ms(step, 0.0);
  for (int64_t q = 0; q < step; ++q) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, opev[2 * q], opev[2 * q + 1]) == hipSuccess) step_ms[q] = ms;
  }
  for (int64_t q = 0; q < step; ++q)
    for (int pi : step_members[q]) E.P[pi].t_op_ms += step_ms[q];
  for (hipEvent_t e : opev) (void)hipEventDestroy(e);

  eda_status first = EDA_OK;
  for (int32_t p = 0; p < count; ++p) {
    BP& P = E.P[p];
    const eda_problem& q = probs[p];
    if (stat[p] == EDA_OK) {
      bool range_err = false;
      for (int64_t i = 0; i < P.t; ++i) {
        const double th = P.theta[i];
        if (!(th > 0.0)) {
          range_err = true;
          q.ritz_log[i] = -INFINITY;
          q.ritz[i] = 0.0;
        } else {
          q.ritz_log[i] = P.sub->shiftB + std::log(th);
          q.ritz[i] = std::exp(q.ritz_log[i]);
        }
        q.resid[i] = (E.resmode == EDA_RES_REL_THETA) ? P.est[i] / th : P.est[i] / P.theta[0];
      }
      if (P.floor_limited) P.flags_out |= EDA_WARN_FLOOR;
      if (P.hfl[0] | P.hfl[1]) P.flags_out |= EDA_WARN_REPAIRED;
      if (range_err)
        stat[p] = EDA_ERR_RANGE;
      else if (!P.converged)
        stat[p] = EDA_ERR_NOCONV;
    }
    // A narrow-precision problem whose refinement stalled (wanted pairs a few
    // per cent from a large eigenvalue cluster) continues in float64 on its
    // own handle: its float64 master becomes the storage (Gram and cores are
    // kept) and block Lanczos starts from the refined Ritz block mixed down
    // to b columns, so the Krylov space begins inside the wanted subspace.
    eda_info fb;
    std::memset(&fb, 0, sizeof(fb));
    bool fell_back = false;
    if (stat[p] == EDA_ERR_NOCONV && E.mixed) {
      eda_status s1 = promote_storage_f64(P.sub);
      double* V1 = nullptr;
      int64_t ld1 = 0;
      if (s1 == EDA_OK)
        s1 = warm_start_block(P.sub, P.d, P.t, E.b, P.XB[P.cb], P.ldq, E.seed + (uint64_t)p, &V1,
                              &ld1);
      if (s1 == EDA_OK) {
        eda_solve_opts o1;
        std::memset(&o1, 0, sizeof(o1));
        o1.form = EDA_FORM_LANCZOS_M;
        o1.block = (int32_t)E.b;
        o1.resmode = E.resmode;
        o1.krylov_dtype = EDA_F64;
        o1.refine_dtype = EDA_F64;
        o1.seed = E.seed + (uint64_t)p;
        o1.start_block = V1;
        o1.ld_start = ld1;
        s1 = eda_solve(P.sub, (int32_t)q.t, q.tol, &o1, q.ritz, q.ritz_log, q.X, q.ldx, q.resid,
                       &fb);
      }
      if (s1 == EDA_OK) {
        stat[p] = EDA_OK;
        fell_back = true;
      }
    }
    if (infos != nullptr) {
      eda_info& I = infos[p];
      std::memset(&I, 0, sizeof(I));
      I.iters = (int32_t)P.iters;
      I.restarts = (int32_t)P.restarts;
      I.refine_passes = (int32_t)P.passes;
      I.flags = P.flags_out;
      I.ops = P.ops;
      I.bytes_moved = P.bytes;
      I.t_prepare_ms = prep_ms;
      I.t_krylov_ms = kry_ms;
      I.t_refine_ms = ref_ms;
      I.shift_s = P.sub->shiftB;
      I.op_calls = P.op_calls;
      I.t_op_ms = P.t_op_ms;
      I.op_bytes = 2.0 * P.d * P.N * dsize(storage) + 3.0 * P.d * b * qs;
      if (fell_back) {  // the float64 continuation's work is part of this problem's
        I.iters += fb.iters;
        I.restarts += fb.restarts;
        I.refine_passes += fb.refine_passes;
        I.flags = fb.flags | EDA_WARN_FALLBACK;
        I.ops += fb.ops;
        I.bytes_moved += fb.bytes_moved;
        I.t_krylov_ms += fb.t_krylov_ms;
        I.t_refine_ms += fb.t_refine_ms;
        I.op_calls += fb.op_calls;
        I.t_op_ms += fb.t_op_ms;
      }
    }
    if (statuses != nullptr) statuses[p] = stat[p];
    if (stat[p] != EDA_OK && first == EDA_OK) first = stat[p];
  }
  if (first != EDA_OK) return fail(h, first, "some problems of the batch did not succeed");
  return EDA_OK;
}
