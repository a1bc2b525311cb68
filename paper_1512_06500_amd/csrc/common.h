// Shared definitions of the libeda HIP sources (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>

namespace eda {

constexpr int kWave = 64;

// ---------------------------------------------------------------------------
// Scalar conversions used by the templated kernels.
// ---------------------------------------------------------------------------
template <typename T> __device__ __forceinline__ double to_f64(T x);
template <> __device__ __forceinline__ double to_f64<double>(double x) { return x; }
template <> __device__ __forceinline__ double to_f64<float>(float x) { return (double)x; }

template <typename T> __device__ __forceinline__ float to_f32(T x);
template <> __device__ __forceinline__ float to_f32<double>(double x) { return (float)x; }
template <> __device__ __forceinline__ float to_f32<float>(float x) { return x; }

template <typename ACC, typename T> __device__ __forceinline__ ACC to_acc(T x);
template <> __device__ __forceinline__ double to_acc<double, double>(double x) { return x; }
template <> __device__ __forceinline__ double to_acc<double, float>(float x) { return (double)x; }
template <> __device__ __forceinline__ float to_acc<float, float>(float x) { return x; }
template <> __device__ __forceinline__ float to_acc<float, double>(double x) { return (float)x; }

template <typename T> __device__ __forceinline__ T from_f64(double x);
template <> __device__ __forceinline__ double from_f64<double>(double x) { return x; }
template <> __device__ __forceinline__ float from_f64<float>(double x) { return (float)x; }

// bfloat16: 8 exponent bits (bias 127), 7 stored mantissa bits.
using bf16_t = __hip_bfloat16;

// Code of the bfloat16 value nearest to x, rounded once from float64 (ties
// to the even significand).  The spacing of bfloat16 values around |x| is a
// power of two 2^qe (2^-133 among the subnormals), so |x| 2^-qe is exact in
// float64 and rint rounds it; magnitudes that round to 2^128 become
// infinity.  (Converting to float first would round twice: a value just
// above a bfloat16 tie can land on the tie in float32 and then go to even.)
__device__ inline uint16_t bf16_bits_rne(double x) {
  if (x != x) return 0x7fc0;
  const uint16_t s = signbit(x) ? 0x8000 : 0;
  const double a = fabs(x);
  if (a == 0.0) return s;
  if (a >= 0x1.0p128) return s | 0x7f80;
  int e;
  (void)frexp(a, &e);  // a in [2^(e-1), 2^e)
  const int qe = ((e - 1 > -126) ? e - 1 : -126) - 7;
  const double r = ldexp(rint(ldexp(a, -qe)), qe);
  if (r >= 0x1.0p128) return s | 0x7f80;
  return s | (uint16_t)(__float_as_uint((float)r) >> 16);  // r is exact in float
}
template <> __device__ __forceinline__ double to_f64<bf16_t>(bf16_t x) {
  return (double)__bfloat162float(x);
}
template <> __device__ __forceinline__ float to_acc<float, bf16_t>(bf16_t x) {
  return __bfloat162float(x);
}
template <> __device__ __forceinline__ double to_acc<double, bf16_t>(bf16_t x) {
  return (double)__bfloat162float(x);
}
template <> __device__ __forceinline__ bf16_t from_f64<bf16_t>(double x) {
  return __ushort_as_bfloat16(bf16_bits_rne(x));
}

// FP8 E4M3 in the OCP layout (sign, 4 exponent bits with bias 7, 3 mantissa
// bits; no infinities, S.1111.111 is NaN, largest finite 448).  Decoding is
// exact; encoding rounds to nearest even and saturates at +-448.
struct fp8e4m3 {
  uint8_t b;
};
__host__ __device__ inline float fp8e4m3_decode(uint8_t b) {
  const uint32_t s = (uint32_t)(b & 0x80u) << 24;
  const uint32_t e = (b >> 3) & 15u, m = b & 7u;
  if (e == 0) {
    const float v = (float)m * 0x1.0p-9f;  // subnormal: m/8 * 2^-6
    return s ? -v : v;
  }
  if (e == 15 && m == 7) return __builtin_nanf("");
  union {
    uint32_t u;
    float f;
  } r;
  r.u = s | ((e + 120u) << 23) | (m << 20);
  return r.f;
}
__device__ inline uint8_t fp8e4m3_encode(double x) {
  if (!(x == x)) return 0x7f;
  const uint8_t s = (x < 0.0) ? 0x80 : 0x00;
  const double a = fabs(x);
  if (a >= 448.0) return s | 0x7e;
  if (a < 0x1.0p-6) return s | (uint8_t)rint(a * 512.0);  // 8 is 2^-6 (exponent 1)
  int e;
  const double f = frexp(a, &e);                // a = f 2^e, f in [0.5, 1)
  double q = rint((2.0 * f - 1.0) * 8.0);       // mantissa, 0 .. 8
  int E = e + 6;                                // biased exponent of 2 f 2^(e-1)
  if (q == 8.0) {
    q = 0.0;
    ++E;
  }
  if (E > 15 || (E == 15 && q > 6.0)) return s | 0x7e;
  return s | (uint8_t)((E << 3) | (int)q);
}
template <> __device__ __forceinline__ double to_f64<fp8e4m3>(fp8e4m3 x) {
  return (double)fp8e4m3_decode(x.b);
}
template <> __device__ __forceinline__ float to_acc<float, fp8e4m3>(fp8e4m3 x) {
  return fp8e4m3_decode(x.b);
}
template <> __device__ __forceinline__ double to_acc<double, fp8e4m3>(fp8e4m3 x) {
  return (double)fp8e4m3_decode(x.b);
}

// ---------------------------------------------------------------------------
// Wave-level exchanges (wave64).
// ---------------------------------------------------------------------------
// Value of v in lane `lane` (the same lane for the whole wave).
__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Lane exchanges within rows of 16 lanes (DPP): partner l^1, l^2 inside a
// quad, the mirror inside 8 lanes (pairs the two quads) and inside 16
// lanes (pairs the two halves).  Every pattern is an involution, so a
// reduction built from them leaves the same bits in both partners.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppMirror8 = 0x141, kDppMirror16 = 0x140;
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes (all active); every lane gets the same bits.
__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_f64<kDppXor1>(v);
  v += dpp_f64<kDppXor2>(v);
  v += dpp_f64<kDppMirror8>(v);
  v += dpp_f64<kDppMirror16>(v);
  return (readlane_f64(v, 0) + readlane_f64(v, 16)) + (readlane_f64(v, 32) + readlane_f64(v, 48));
}

// Standard normal sample for element e of a seeded stream: two SplitMix64
// outputs (Steele, Lea, Flood 2014) turned into one Box-Muller deviate.
__device__ __forceinline__ double masked_gauss(uint64_t seed, int64_t e) {
  uint64_t z1 = (seed ^ 0x2545f4914f6cdd1dull) + 2ull * (uint64_t)e * 0x9e3779b97f4a7c15ull;
  uint64_t z2 = z1 + 0x9e3779b97f4a7c15ull;
  z1 = (z1 ^ (z1 >> 30)) * 0xbf58476d1ce4e5b9ull;
  z1 = (z1 ^ (z1 >> 27)) * 0x94d049bb133111ebull;
  z1 ^= z1 >> 31;
  z2 = (z2 ^ (z2 >> 30)) * 0xbf58476d1ce4e5b9ull;
  z2 = (z2 ^ (z2 >> 27)) * 0x94d049bb133111ebull;
  z2 ^= z2 >> 31;
  const double u1 = ((double)(z1 >> 11) + 1.0) * 0x1.0p-53;
  const double u2 = (double)(z2 >> 11) * 0x1.0p-53;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

// ---------------------------------------------------------------------------
// Host-side launchers (implemented in the .hip files, called by the host sources).
// All take the stream last and return hipError_t of the launch.
// Shapes are validated by the caller; each launcher documents what it needs.
// ---------------------------------------------------------------------------

enum class DT : int { F64 = 0, F32 = 1, BF16 = 2, FP8 = 3 };

// ---------------------------------------------------------------------------
// Multi-problem launches.  Each kernel below exists once and takes its
// arguments as a struct: either by value (one problem) or as a device array
// indexed by blockIdx.z (one entry per problem, sizes may differ; the grid
// covers the largest entry and surplus workgroups of smaller ones exit).
// launch_*_multi(count, host, dev, s): `host` holds the count entries (used
// for the grid, and passed by value when count == 1); `dev` is the same
// array already resident on the device (may be null when count == 1).
// ---------------------------------------------------------------------------
struct TnArgs {      // part[(c * m + i) * nb + j] = sum over chunk c of A(r, i) B(r, j)
  int64_t d, m, nb, lda, ldb, chunks;
  const void* A;
  const void* B;
  double* part;
  const int* gate;
  const double* ascale;  // when not null, column i of A is scaled by ascale[i] (FP8 storage)
};
struct ReduceArgs {  // C = beta C + alpha sum_c part (col-major), Z = zalpha sum (row-major)
  int64_t chunks, m, nb, ldc, ldz;
  const double* part;
  double alpha, beta, zalpha;
  double* C;
  double* Z;
  const int* gate;
  // when mc >= 0, rows i >= mc go to C2[(i - mc) + j*ldc2] (plain sum) instead of C
  int64_t mc = -1, ldc2 = 0;
  double* C2 = nullptr;
};
struct NnArgs {      // Out = alpha V + A Z
  int64_t d, m, nb, lda, ldz, ldv, ldo;
  const void* A;
  const double* Z;
  double alpha;
  const void* V;
  void* Out;
  int out_row;
  const int* gate;
  const double* alpha_p;  // when not null, alpha is read from here (device)
  const double* ascale;   // when not null, column i of A is scaled by ascale[i] (FP8 storage)
  const int* mask;        // when not null, output columns j with mask[j] != 0 get
  uint64_t seed;          //   masked_gauss(seed, j * d + row) instead of the product
  // when > 0: column groups of kcols columns, each writing its partial
  // product row-major to Out + group * d * nb (streaming kernel only)
  int64_t kcols = 0;
};
struct CholArgs {
  int64_t b, ldg, ldri, ldrp, ldro, m, ldhc;
  const double* G;
  double* Rinv;
  const double* Rprev;
  double* Rout;
  const double* hcol;
  double ratio;
  int* flag;
  const int* gate;
  const double* part;  // when not null, G = sum over `chunks` tn partials (layout of tn, m = nb = b)
  int64_t chunks;
};
struct PcholArgs {
  int64_t b, ldg, m, ldhc, ldz, ldr;
  const double* G;
  const double* hcol;
  double tau, ratio;
  int equil;
  double* Z;
  double* R;
  int* mask;
  int* flag;
  const double* part;  // when not null, G = sum over `chunks` tn partials (layout of tn, m = nb = b)
  int64_t chunks;
  // when not null, G -= corr^T corr (corr row-major mcorr x b)
  const double* corr = nullptr;
  int64_t mcorr = 0;
};
struct MaskedRandnArgs {  // Q[:, j] = seeded Gaussian where mask[j] != 0
  int64_t d, b, ldq;
  const int* mask;
  uint64_t seed;
  void* Q;
};
struct RandnArgs { int64_t d, b, ldv; uint64_t seed; double* V; };
struct Copy2dArgs { int64_t rows, cols, lds, ldd; const void* src; void* dst; };
struct FillArgs { int64_t count; double v; double* dst; };
struct FillI32Args { int64_t count; int v; int* dst; };
struct SymArgs { int64_t m, ldh, ldt; const double* H; double* T; };
struct RitzEstArgs {
  int64_t m, b, cnt, lds, ldbm;
  const double* w;
  const double* S;
  const double* Bm;
  double* th;
  double* res;
};
struct GatherArgs { int64_t m, cnt, lds, ldsd; const double* S; double* Sd; };
struct SetDiagArgs { int64_t cnt, ldd; const double* v; double* D; };
struct CouplingArgs {
  int64_t m, b, kk, ldbm, ldsd, ldh;
  const double* Bm;
  const double* Sd;
  double* Hn;
};
struct ResidArgs {
  int64_t d, t, ldmy, ldy, ldr;
  const double* MY;
  const double* Y;
  const double* theta;
  double* R;
  double* res;
};
struct DescArgs { int64_t cnt, n; const double* w; double* out; };
struct SignArgs { int64_t d, t, ldx; double* X; };
struct FlagArgs { int* flags; };
struct SyevArgs {    // one symmetric eigenproblem, see launch_syev
  int64_t n, lda, ldz, nvec;
  const double* A;
  double* w;
  double* Z;
  double* work;
  double ctol = 0.0;  // cluster gap relative to ||T|| (0: orthonormal, see launch_syev)
};

// Kernel-side selection of the argument source of a multi launch.
template <typename A>
inline void pick(int count, const A* host, const A* dev, const A** arr, A* one) {
  *arr = (count == 1) ? nullptr : dev;
  *one = (count == 1) ? host[0] : A{};
}

hipError_t launch_tn_multi(int count, const TnArgs* host, const TnArgs* dev, DT adt, DT bdt,
                           hipStream_t s);
hipError_t launch_reduce_multi(int count, const ReduceArgs* host, const ReduceArgs* dev,
                               hipStream_t s);
hipError_t launch_nn_multi(int count, const NnArgs* host, const NnArgs* dev, DT adt, DT vdt,
                           DT odt, hipStream_t s);
hipError_t launch_chol_multi(int count, const CholArgs* host, const CholArgs* dev, hipStream_t s);
hipError_t launch_pchol_multi(int count, const PcholArgs* host, const PcholArgs* dev,
                              hipStream_t s);
hipError_t launch_masked_randn_multi(int count, const MaskedRandnArgs* host,
                                     const MaskedRandnArgs* dev, DT qdt, hipStream_t s);
hipError_t launch_randn_multi(int count, const RandnArgs* host, const RandnArgs* dev,
                              hipStream_t s);
hipError_t launch_copy2d_multi(int count, const Copy2dArgs* host, const Copy2dArgs* dev, DT sdt,
                               DT ddt, hipStream_t s);
hipError_t launch_fill_multi(int count, const FillArgs* host, const FillArgs* dev, hipStream_t s);
hipError_t launch_fill_i32_multi(int count, const FillI32Args* host, const FillI32Args* dev,
                                 hipStream_t s);
hipError_t launch_symmetrize_multi(int count, const SymArgs* host, const SymArgs* dev,
                                   hipStream_t s);
hipError_t launch_ritz_estimates_multi(int count, const RitzEstArgs* host, const RitzEstArgs* dev,
                                       hipStream_t s);
hipError_t launch_gather_desc_multi(int count, const GatherArgs* host, const GatherArgs* dev,
                                    hipStream_t s);
hipError_t launch_set_diag_multi(int count, const SetDiagArgs* host, const SetDiagArgs* dev,
                                 hipStream_t s);
hipError_t launch_restart_coupling_multi(int count, const CouplingArgs* host,
                                         const CouplingArgs* dev, hipStream_t s);
hipError_t launch_ritz_residual_multi(int count, const ResidArgs* host, const ResidArgs* dev,
                                      hipStream_t s);
hipError_t launch_desc_values_multi(int count, const DescArgs* host, const DescArgs* dev,
                                    hipStream_t s);
hipError_t launch_sign_fix_multi(int count, const SignArgs* host, const SignArgs* dev,
                                 hipStream_t s);
hipError_t launch_flag_fold_multi(int count, const FlagArgs* host, const FlagArgs* dev,
                                  hipStream_t s);
hipError_t launch_syev_multi(int count, const SyevArgs* host, const SyevArgs* dev,
                             hipStream_t s);
// Chunk count of a tn launch for one entry (the step count S is chosen from
// the largest d and m of the launch, so pass those).
int64_t tn_chunks_for(int64_t d, int64_t dmax, int64_t mmax);

// k_basic.hip ---------------------------------------------------------------
// H_W, H_B from class-contiguous samples (counts given as offsets[k+1] on device).
hipError_t launch_scatter(int64_t d, int64_t n, int64_t k, const double* X, int64_t ldx,
                          const int64_t* offsets, double* H_W, int64_t ldw, double* H_B,
                          int64_t ldb, hipStream_t s);
// P[:, col0:col0+cols] = cast(H) for rows < d, zero for d <= row < ldp.
// FP8 copy of the float64 matrix P64 (ld ldp, cols columns): scale[j] =
// max |P64[:, j]| / 448, P8[r, j] = E4M3(P64[r, j] / scale[j]), rows d..ldp-1 zero.
hipError_t launch_pack_fp8(int64_t d, int64_t ldp, int64_t cols, const double* P64,
                           double* scale, void* P8, hipStream_t s);
// P[:, col0 .. col0 + cols) (ld ldp, rows d .. ldp-1 zero) = H in type pdt;
// with a flag, flag[0] |= 1 if any entry of H is NaN/Inf.
hipError_t launch_pack(int64_t d, int64_t ldp, int64_t cols, const double* H, int64_t ldh,
                       void* P, DT pdt, int64_t col0, hipStream_t s, int* flag = nullptr);
// flag[0] |= 1 if any entry of the d x cols matrix is NaN/Inf.
hipError_t launch_nonfinite(int64_t d, int64_t cols, const double* H, int64_t ldh, int* flag,
                            hipStream_t s);
// Seeded Gaussian d x b block (SplitMix64 counter hash + Box-Muller), float64.
hipError_t launch_randn(int64_t d, int64_t b, uint64_t seed, double* V, int64_t ldv,
                        hipStream_t s);
// Dst (rows x cols, type dt) = Src (rows x cols, float64 or same dt).
hipError_t launch_copy2d(int64_t rows, int64_t cols, const void* src, DT sdt, int64_t lds,
                         void* dst, DT ddt, int64_t ldd, hipStream_t s);
// f[i] = phi-type weights for a core: see k_basic.hip.
hipError_t launch_core_weights(int64_t n, const double* lam, double c, double shift, double* f,
                               hipStream_t s);
// dst[r + c*ldd] = alpha * (trans ? src[c + r*lds] : src[r + c*lds]), rows x cols of dst.
hipError_t launch_copy_block(int64_t rows, int64_t cols, double alpha, const double* src,
                             int64_t lds, bool trans, double* dst, int64_t ldd, hipStream_t s);
// out[0] = max_j sum_i |A[i + j*lda]| (1-norm of an n x n matrix).
hipError_t launch_norm1(int64_t n, const double* A, int64_t lda, double* out, hipStream_t s);
// C = a0 I + a1 X1 + a2 X2 + a3 X3 (n x n; X2/X3 may be null when a2/a3 are 0).
hipError_t launch_lincomb(int64_t n, double a0, double a1, const double* X1, double a2,
                          const double* X2, double a3, const double* X3, int64_t ldx,
                          double* C, int64_t ldc, hipStream_t s);
// dst[r + c*ldd] = src[r + c*lds] * w[c]^(p/2), p = +1 or -1 (columns scaled
// by the square roots of w, or their reciprocals).
hipError_t launch_scale_cols(int64_t rows, int64_t cols, const double* src, int64_t lds,
                             const double* w, int p, double* dst, int64_t ldd, hipStream_t s);
// dst[i + i*ldd] = v[i] for i < cnt (diagonal only).
hipError_t launch_set_diag(int64_t cnt, const double* v, double* dst, int64_t ldd, hipStream_t s);
// Column 2-norms / sign fix / scaling helpers.
hipError_t launch_sign_fix(int64_t d, int64_t t, double* X, int64_t ldx, hipStream_t s);
// 1-NN in a t-dimensional projection: for every testing row j of Pte
// (row-major n_test x t) the training row i of Ptr (row-major n_train x t)
// with the smallest ||Ptr_i - Pte_j||_2 (ties: the smallest i).
hipError_t launch_nn_classify(int64_t n_train, int64_t n_test, int64_t t, const double* Ptr,
                              const double* Pte, const int32_t* labels, int32_t* pred,
                              int64_t* idx, double* dist, hipStream_t s);
hipError_t launch_fill(int64_t count, double value, double* dst, hipStream_t s);
hipError_t launch_fill_i32(int64_t count, int value, int* dst, hipStream_t s);
// Symmetrised copy T = (H[0:m,0:m] + H[0:m,0:m]^T)/2.
hipError_t launch_symmetrize(int64_t m, const double* H, int64_t ldh, double* T, int64_t ldt,
                             hipStream_t s);
// Ritz diagnostics: theta (top `cnt` of w ascending, returned descending) and
// residual estimates ||Bm * S[m-b:m, i]|| for those pairs.
hipError_t launch_ritz_estimates(int64_t m, int64_t b, int64_t cnt, const double* w,
                                 const double* S, int64_t lds, const double* Bm, int64_t ldbm,
                                 double* out_theta, double* out_res, hipStream_t s);
// Gather eigenvector columns in descending order, row-major: Sd[r*ldsd + i] = S[r + (m-1-i)*lds].
hipError_t launch_gather_desc(int64_t m, int64_t cnt, const double* S, int64_t lds, double* Sd,
                              int64_t ldsd, hipStream_t s);
// flags[1] |= flags[0]; flags[0] = 0.
hipError_t launch_flag_fold(int* flags, hipStream_t s);
// R(:, i) = MY(:, i) - theta_i Y(:, i) (stored when R != null); res[i] = ||R(:, i)||.
hipError_t launch_ritz_residual(int64_t d, int64_t t, const double* MY, int64_t ldmy,
                                const double* Y, int64_t ldy, const double* theta, double* R,
                                int64_t ldr, double* res, hipStream_t s);
// out[i] = w[n - 1 - i] for i < cnt.
hipError_t launch_desc_values(int64_t cnt, const double* w, int64_t n, double* out,
                              hipStream_t s);
// Restart coupling: Hn[kk + r, c] = sum_q Bm[r, q] * S[m - b + q, c] for c < kk.
hipError_t launch_restart_coupling(int64_t m, int64_t b, int64_t kk, const double* Bm,
                                   int64_t ldbm, const double* Sd, int64_t ldsd, double* Hn,
                                   int64_t ldh, hipStream_t s);

// Tile table (eda_tune.cpp): tuned launch shapes per shape class
// (kind, ceil(log2 d), ceil(log2 m), entry bytes); -1 when not tuned.
//   TnSteps: 64-row steps per wave of the tn kernel (1, 2, 4 or 8), which fixes
//            its chunk count (tn_chunks); NnTile: nn configuration index
//            0 (16 rows, 4 loads per batch), 1 (16, 16), 2 (32, 8), 3 (64, 8).
enum class TuneKind { TnSteps = 0, NnTile = 1 };
constexpr int kNnConfigs = 4;
int tune_get(TuneKind kind, int64_t d, int64_t m, int esize);
void tune_set(TuneKind kind, int64_t d, int64_t m, int esize, int value);

// k_tsmm.hip ----------------------------------------------------------------
// Partial sums of A^T B over row chunks: part[(c*m + i)*nb + j], c < chunks.
// Returns the number of chunks used through *chunks_out (computed from shape).
int64_t tn_chunks(int64_t d, int64_t m, int64_t nb);
hipError_t launch_tn_partial(int64_t d, int64_t m, int64_t nb, const void* A, DT adt,
                             int64_t lda, const void* B, DT bdt, int64_t ldb, double* part,
                             int64_t chunks, const int* gate, hipStream_t s,
                             const double* ascale = nullptr);
// C_col[i + j*ldc] = beta*C_col + alpha*sum_c part  (if C_col != null)
// Z_row[i*ldz + j] = zalpha*sum_c part              (if Z_row != null)
// (with mc >= 0: rows i >= mc go to C2[(i - mc) + j*ldc2] = sum_c part instead)
hipError_t launch_reduce_partials(int64_t chunks, int64_t m, int64_t nb, const double* part,
                                  double alpha, double beta, double* C_col, int64_t ldc,
                                  double zalpha, double* Z_row, int64_t ldz, const int* gate,
                                  hipStream_t s, int64_t mc = -1, double* C2 = nullptr,
                                  int64_t ldc2 = 0);
// Out = alpha * V + A * Z, Z row-major (Z[i*ldz + j]) float64, m columns of A.
// Out column-major (Out[r + j*ldo]) or, with out_row, row-major (Out[r*ldo + j]).
// Z = C Y for a square float64 C (m x m, column-major ldc) and a row-major
// float64 Y (m x nb, nb <= 8, ld ldy): the columns of C are split into
// groups whose partial products are written to `part` (at least
// nn_split_groups(m) * m * nb doubles) and summed in a fixed order into Z
// (row-major, ld ldz).  Returns hipErrorInvalidValue when the shape does not
// suit the split (the caller then uses launch_nn).
int64_t nn_split_groups(int64_t m);
// k_jd.hip: the lockstep GMRES of the Jacobi-Davidson inner solve (c <= 64
// columns, k <= 8 steps; H: c Hessenberg matrices of (k+1) x k, see there).
hipError_t launch_jd_gs_coeffs(int blocks, int c, int k, int l, const double* G, double* D,
                               double* H, hipStream_t s);
hipError_t launch_jd_norms(int c, int k, int l, const double* G, double tiny, double* S,
                           double* H, hipStream_t s);
hipError_t launch_jd_gmres_ls(int c, int k, const double* H, const double* beta, double* Y,
                              hipStream_t s);
// Out = alpha V + A Z for a narrow A (bfloat16 or FP8 codes, d x m, lda a
// multiple of 8, column scales ascale or null) and nb <= 8: column groups
// of A write float32 partial rows to `part` (at least
// nn_narrow_split_groups(d, m) * d * 8 floats, 16-byte aligned), summed in a
// fixed order by a second kernel that adds alpha V (alpha from alpha_p when
// not null) and rounds to odt (== vdt, float32 or bfloat16: the sums are
// float32).  hipErrorInvalidValue when the shape does not suit it (the
// caller then uses launch_nn).
int64_t nn_narrow_split_groups(int64_t d, int64_t m);
hipError_t launch_nn_narrow_split(int64_t d, int64_t m, int64_t nb, const void* A, DT adt,
                                  int64_t lda, const double* Z, int64_t ldz, double alpha,
                                  const double* alpha_p, const void* V, DT vdt, int64_t ldv,
                                  void* Out, DT odt, int64_t ldo, const double* ascale,
                                  float* part, hipStream_t s);
hipError_t launch_nn_split(int64_t m, int64_t nb, const double* C, int64_t ldc, const double* Y,
                           int64_t ldy, double* part, double* Z, int64_t ldz, hipStream_t s);
hipError_t launch_nn(int64_t d, int64_t m, int64_t nb, const void* A, DT adt, int64_t lda,
                     const double* Z, int64_t ldz, double alpha, const void* V, DT vdt,
                     int64_t ldv, void* Out, DT odt, int64_t ldo, const int* gate,
                     hipStream_t s, bool out_row = false, const double* alpha_p = nullptr,
                     const double* ascale = nullptr, const int* mask = nullptr,
                     uint64_t seed = 0);

// k_gemm.hip ----------------------------------------------------------------
// C (m x n) = alpha * op(A) * diag(dk) * op(B) + beta * C, float64, col-major.
// op(X) = X or X^T; dk may be null (identity).
hipError_t launch_gemm(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double alpha,
                       const double* A, int64_t lda, const double* dk, const double* B,
                       int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s);
// The same for an n x n product the caller knows to be symmetric (with
// beta != 0, C symmetric too): only the lower triangle is computed, then
// mirrored, so the result is exactly symmetric (large n; small n falls back
// to launch_gemm).
// C = A Z + gv V (gv from gv_p when not null; V may be null) on the matrix
// cores in 64 x 64 tiles: A m x k column-major, Z k x n row-major (Z(r, j) at
// Z[r ldz + j]), V and C m x n column-major.  Requires k >= 16, an even lda
// and a 16-byte aligned A (hipErrorInvalidValue otherwise).
hipError_t launch_gemm_av(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                          const double* Z, int64_t ldz, double gv, const double* gv_p,
                          const double* V, int64_t ldv, double* C, int64_t ldc, hipStream_t s);
// C = alpha op(A) op(B) + beta C for an n x n result known to be symmetric
// (lower tiles computed, mirrored).  ws (ws_bytes; may be null) holds the
// partial tiles when the tiles are split along K, which needs
// gemm_sym_ws_bytes(n, k) bytes (0: no split); calls sharing ws must be
// ordered (one stream).
hipError_t launch_gemm_sym(bool ta, bool tb, int64_t n, int64_t k, double alpha, const double* A,
                           int64_t lda, const double* dk, const double* B, int64_t ldb,
                           double beta, double* C, int64_t ldc, hipStream_t s,
                           double* ws = nullptr, int64_t ws_bytes = 0);
int64_t gemm_sym_ws_bytes(int64_t n, int64_t k);
// G = X^T X (N x N, ld ldg, exactly symmetric) of a float64 d x N block with
// 16-byte aligned columns and an even ld, on the matrix cores; part holds
// gram_block_chunks(d, N) partial N x N matrices.
int64_t gram_block_chunks(int64_t d, int64_t N);
hipError_t launch_gram_block(int64_t d, int64_t N, const double* X, int64_t ldx, double* part,
                             int64_t chunks, double* G, int64_t ldg, hipStream_t s);
// Gram partials: part[c][i][j] over lower-triangle tiles; finalised by launch_gram_reduce.
int64_t gram_chunks(int64_t d, int64_t N);
hipError_t launch_gram_partial(int64_t d, int64_t N, const void* P, DT pdt, int64_t ldp,
                               double* part, int64_t chunks, hipStream_t s);
hipError_t launch_gram_reduce(int64_t N, int64_t chunks, const double* part, double* G,
                              int64_t ldg, hipStream_t s);

// k_chol.hip ----------------------------------------------------------------
// Cholesky G = R^T R (b x b), outputs R^{-1} row-major (Rinv[i*ldri + j]) and,
// if Rout != null, Rout = R * Rprev (or R when Rprev is null), col-major.
// If hcol != null, sets *flag = 1 when some column kept less than `ratio` of
// its norm through the projection (hcol: m x b projection coefficients).
// With part != null, G is the fixed-order sum of the `chunks` tn partials
// part[(c*b + i)*b + j] (G and ldg unused).
hipError_t launch_chol(int64_t b, const double* G, int64_t ldg, double* Rinv, int64_t ldri,
                       const double* Rprev, int64_t ldrp, double* Rout, int64_t ldro,
                       const double* hcol, int64_t m, int64_t ldhc, double ratio, int* flag,
                       const int* gate, hipStream_t s, const double* part = nullptr,
                       int64_t chunks = 0);

// Rank-revealing pivoted Cholesky of a Lanczos block (b <= 64); see k_chol.hip.
// With `equil`, the block is first scaled to unit column norms (hcol ignored)
// and the scaling is folded back into Z and R.
hipError_t launch_pchol(int64_t b, const double* G, int64_t ldg, const double* hcol, int64_t m,
                        int64_t ldhc, double tau, double ratio, bool equil, double* Z, int64_t ldz,
                        double* R, int64_t ldr, int* mask, int* flag, hipStream_t s,
                        const double* part = nullptr, int64_t chunks = 0,
                        const double* corr = nullptr, int64_t mcorr = 0);
// Q[:, j] = seeded Gaussian for the columns with mask[j] != 0.
hipError_t launch_fill_masked_randn(int64_t d, int64_t b, const int* mask, uint64_t seed,
                                    void* Q, DT qdt, int64_t ldq, hipStream_t s);

// k_syev.hip ----------------------------------------------------------------
// Batched symmetric eigensolver, one workgroup per matrix. For matrix q:
//   A_q at A + q*strideA (lda), w_q at w + q*stridew, Z_q at Z + q*strideZ (ldz).
// n_q = ns[q] (device int array) or n when ns is null.  Eigenvalues ascending;
// only the top nvec_q = min(nvec, n_q) eigenvalues (nvec <= 0: all) are
// computed (the others are returned as 0), with their eigenvectors in columns
// n_q-nvec_q .. n_q-1 of Z_q.
size_t syev_work_bytes(int64_t nmax);
void syev_timing_enable(bool on);
void syev_timing_report(FILE* f);
// ctol <= 0: eigenvectors orthonormal to working accuracy (clusters of gaps
// up to 1e-8 ||T|| orthonormalised together, then a correction of the whole
// block).  ctol > 0: only clusters of gaps up to ctol ||T|| are
// orthonormalised, for callers that need the vectors orthogonal to no better
// than about u / ctol.
hipError_t launch_syev(int64_t batch, int64_t n, const int* ns, const double* A, int64_t lda,
                       int64_t strideA, double* w, int64_t stridew, double* Z, int64_t ldz,
                       int64_t strideZ, int64_t nvec, double* work, hipStream_t s,
                       double ctol = 0.0);

}  // namespace eda
