// Dense FP64 products: general GEMM for the cores (n x n and n x k factors
// of the exponentials) and the Gram matrix P^T P of the scatter factors, on
// the matrix cores (128 x 128 tiles for large shapes, 32 x 32 for small
// ones), plus a register-tiled FMA Gram kernel for narrow factors.
#include <algorithm>
#include <atomic>

#include "common.h"

namespace eda {

namespace {

constexpr int GT = 64;   // tile edge
constexpr int GK = 16;   // K slice

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int MT = 32;  // output tile edge of the matrix-core GEMM
constexpr int MK = 64;  // K slice

// C = alpha op(A) diag(dk) op(B) + beta C on the matrix cores: a 256-thread
// workgroup owns a 32 x 32 tile of C, each wave one 16 x 16 block of it,
// accumulated by v_mfma_f64_16x16x4f64 over K slices of 64 staged in LDS.
// The next slice is loaded into registers while the current one is
// multiplied, so a slice costs one memory round trip at most (the products
// of the cores have K = n or k, a few slices).  Operand lane layout:
// A(i, k) at lane i + 16 k, B(k, j) at lane j + 16 k; accumulator element v
// of lane l is C(4 v + l / 16, l % 16).
__global__ __launch_bounds__(256) void gemm_kernel(bool ta, bool tb, int64_t m, int64_t n, int64_t k,
                                                   double alpha, const double* __restrict__ A,
                                                   int64_t lda, const double* __restrict__ dk,
                                                   const double* __restrict__ B, int64_t ldb,
                                                   double beta, double* __restrict__ C,
                                                   int64_t ldc) {
  __shared__ double As[MT][MK + 1];  // op(A)(i, k)
  __shared__ double Bs[MK][MT + 1];  // op(B)(k, j)
  constexpr int NL = MT * MK / 256;  // elements of each tile per thread
  const int tid = threadIdx.x;
  const int lane = tid & 63, wid = tid >> 6;
  const int64_t i0 = blockIdx.x * (int64_t)MT, j0 = blockIdx.y * (int64_t)MT;
  const int bi = (wid >> 1) * 16, bj = (wid & 1) * 16;
  // element q of this thread: (ii, kk) of op(A) and (kb, jj) of op(B), with
  // consecutive threads on consecutive addresses
  auto a_pos = [&](int q, int& ii, int& kk) {
    const int e = tid + q * 256;
    if (!ta) { ii = e & (MT - 1); kk = e / MT; } else { kk = e & (MK - 1); ii = e / MK; }
  };
  auto b_pos = [&](int q, int& kb, int& jj) {
    const int e = tid + q * 256;
    if (!tb) { kb = e & (MK - 1); jj = e / MK; } else { jj = e & (MT - 1); kb = e / MT; }
  };
  double ra[NL], rb[NL];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      int ii, kk, kb, jj;
      a_pos(q, ii, kk);
      b_pos(q, kb, jj);
      const int64_t gi = i0 + ii, gk = k0 + kk, gj = j0 + jj, gk2 = k0 + kb;
      double v = 0.0, w = 0.0;
      if (gi < m && gk < k) {
        v = ta ? A[gk + gi * lda] : A[gi + gk * lda];
        if (dk != nullptr) v *= dk[gk];
      }
      if (gj < n && gk2 < k) w = tb ? B[gj + gk2 * ldb] : B[gk2 + gj * ldb];
      ra[q] = v;
      rb[q] = w;
    }
  };
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  if (k > 0) load(0);
  for (int64_t k0 = 0; k0 < k; k0 += MK) {
    __syncthreads();  // the previous slice has been read
#pragma unroll
    for (int q = 0; q < NL; ++q) {
      int ii, kk, kb, jj;
      a_pos(q, ii, kk);
      b_pos(q, kb, jj);
      As[ii][kk] = ra[q];
      Bs[kb][jj] = rb[q];
    }
    __syncthreads();
    if (k0 + MK < k) load(k0 + MK);  // in flight during the products below
    const int kl = (k - k0 < MK) ? (int)(k - k0) : MK;
#pragma unroll
    for (int ks = 0; ks < MK; ks += 4) {
      if (ks >= kl) break;  // uniform
      const double a = As[bi + (lane & 15)][ks + (lane >> 4)];
      const double b = Bs[ks + (lane >> 4)][bj + (lane & 15)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
  }
  const int64_t gj = j0 + bj + (lane & 15);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int64_t gi = i0 + bi + 4 * v + (lane >> 4);
    if (gi >= m || gj >= n) continue;
    double* cp = C + gi + gj * ldc;
    *cp = (beta == 0.0 ? 0.0 : beta * *cp) + alpha * acc[v];
  }
}

// Large products on the matrix cores: C (M x N) = alpha op(A) diag(dk) op(B)
// (+ beta C), or, for the Gram matrix, partial tiles of P^T P over row
// chunks.  A workgroup owns a BT x BT tile of C (BT = 64): its 4 waves a
// 2 x 2 grid of 32 x 32 quadrants, 4 v_mfma_f64_16x16x4f64 accumulators
// each, so every A or B fragment read from LDS feeds 2 products (128-edge
// tiles, 16 accumulators a wave, need more registers than two waves per
// SIMD leave and spill).  K is
// staged through LDS in slices of BK = 16, op(A) and op(B) both k-major
// (As[k][i], Bs[k][j]: the 16 lanes of a fragment read 128 contiguous bytes),
// and the next slice is loaded into registers with 16-byte loads while the
// current one is multiplied.  Global loads run along whichever index is
// contiguous in memory (i for op(A) = A, k for op(A) = A^T; likewise for B).
// Requires even leading dimensions and 16-byte aligned operands (the
// launcher falls back to gemm_kernel otherwise).
constexpr int BT = 64;  // tile edge of the Gram kernel and of large GEMMs
constexpr int BK = 16;

// LDS row stride (doubles) for a tile edge T: T + 18 for 128, T + 2 for 64,
// both = 2 (mod 16), which keeps the transposing stores (8 lanes on rows 0,
// 2, .., 14 of one column) on distinct banks while the 4 k groups of a
// fragment read nearly disjoint bank ranges
template <int T> struct BigStride { static constexpr int v = (T == 128) ? 146 : 66; };

struct BigGemmArgs {
  int64_t M, N, K, lda, ldb, ldc;
  const double* A;
  const double* B;
  const double* dk;
  double* C;
  double alpha, beta;
  int ta, tb;
  // Gram mode: lower-triangle tiles (blockIdx.x enumerates them), K split
  // into chunks of kchunk rows (blockIdx.y), partial tile written to
  // part + chunk * N * N (column-major N x N, only the tile's entries)
  int gram;
  int64_t kchunk;
  double* part;
  // symmetric mode (M == N, the caller guarantees a symmetric result and,
  // with beta != 0, a symmetric C): lower-triangle tiles only (blockIdx.x
  // enumerates them), full K, every entry i >= j written to C(i, j) and
  // C(j, i), so the result is exactly symmetric
  int sym = 0;
  // general mode with V: C = alpha op(A) op(B) + gv V (V column-major, ldv;
  // gv read from gv_p when that is not null); beta is then unused
  const double* V = nullptr;
  int64_t ldv = 0;
  double gv = 0.0;
  const double* gv_p = nullptr;
  // 0: B is read one double at a time (odd ldb or 8-byte aligned B)
  int b_pairs = 1;
  // symmetric mode with split tiles (nfull >= 0): blockIdx.x < nfull
  // computes tile blockIdx.x whole; blockIdx.x = nfull + u computes K part
  // u % ksplit (kpart rows) of tile nfull + u / ksplit and writes that
  // partial tile to spart + u T T (column-major in the tile); a fixed-order
  // reduction (big_sym_split_reduce_kernel) finishes the split tiles
  int64_t nfull = -1;
  int64_t ksplit = 1;
  int64_t kpart = 0;
  double* spart = nullptr;
};

// Loads of one BK slice of op(X) (rows: the T-edge tile index, k: the
// slice), T BK / 512 pairs of doubles per thread.  trans == false: X(i, k)
// at X[i + k ld] (pairs along i); trans: X(i, k) at X[k + i ld] (pairs
// along k).
template <int T, int NT, bool TRANS>
__device__ __forceinline__ void big_load(const double* __restrict__ X, int64_t ld, bool pairs,
                                         int64_t i0, int64_t nI, int64_t k0, int64_t kend,
                                         double2 (&r)[T * BK / (2 * NT)]) {
  const int tid = threadIdx.x;
  // a slice inside the matrix with 16-byte pairs (wave-uniform test): plain
  // loads, no per-element bounds
  if (pairs && i0 + T <= nI && k0 + BK <= kend) {
#pragma unroll
    for (int q = 0; q < T * BK / (2 * NT); ++q) {
      const int e = tid + NT * q;
      int ii, kk;
      if (!TRANS) { ii = 2 * (e % (T / 2)); kk = e / (T / 2); }
      else { kk = 2 * (e % (BK / 2)); ii = e / (BK / 2); }
      const double* p = TRANS ? X + (k0 + kk) + (i0 + ii) * ld : X + (i0 + ii) + (k0 + kk) * ld;
      r[q] = *(const double2*)p;
    }
    return;
  }
#pragma unroll
  for (int q = 0; q < T * BK / (2 * NT); ++q) {
    const int e = tid + NT * q;
    int ii, kk;
    if (!TRANS) { ii = 2 * (e % (T / 2)); kk = e / (T / 2); }
    else { kk = 2 * (e % (BK / 2)); ii = e / (BK / 2); }
    const int64_t gi = i0 + ii, gk = k0 + kk;
    double2 v = {0.0, 0.0};
    if (!TRANS) {
      if (gk < kend) {
        const double* p = X + gi + gk * ld;
        if (gi + 1 < nI) {
          if (pairs) v = *(const double2*)p;
          else { v.x = p[0]; v.y = p[1]; }
        } else if (gi < nI) {
          v.x = p[0];
        }
      }
    } else {
      if (gi < nI) {
        const double* p = X + gk + gi * ld;
        if (gk + 1 < kend) {
          if (pairs) v = *(const double2*)p;
          else { v.x = p[0]; v.y = p[1]; }
        } else if (gk < kend) {
          v.x = p[0];
        }
      }
    }
    r[q] = v;
  }
}

template <int T, int NT, bool TRANS>
__device__ __forceinline__ void big_store(double (*S)[BigStride<T>::v],
                                          const double2 (&r)[T * BK / (2 * NT)],
                                          const double* __restrict__ dk, int64_t k0,
                                          int64_t kend) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < T * BK / (2 * NT); ++q) {
    const int e = tid + NT * q;
    int ii, kk;
    if (!TRANS) { ii = 2 * (e % (T / 2)); kk = e / (T / 2); }
    else { kk = 2 * (e % (BK / 2)); ii = e / (BK / 2); }
    double x = r[q].x, y = r[q].y;
    if (!TRANS) {
      if (dk != nullptr && k0 + kk < kend) { const double f = dk[k0 + kk]; x *= f; y *= f; }
      S[kk][ii] = x;
      S[kk][ii + 1] = y;
    } else {
      if (dk != nullptr) {
        if (k0 + kk < kend) x *= dk[k0 + kk];
        if (k0 + kk + 1 < kend) y *= dk[k0 + kk + 1];
      }
      S[kk][ii] = x;
      S[kk + 1][ii] = y;
    }
  }
}

// T x T tile per workgroup of NT threads (NW = NT / 64 waves in a 2 x NW/2
// grid); each wave owns a (T/2) x (2T/NW) block of QBI x QBJ MFMA blocks.
template <int T, int NT, bool AT, bool BT_>
__global__ __launch_bounds__(NT, 2) void big_gemm_kernel(BigGemmArgs a) {
  // AT: op(A) = A^T (ta); BT_: B read as X(j, k) along k (tb == 0)
  constexpr int LS = BigStride<T>::v;
  constexpr int NW = NT / 64, WJ = NW / 2;
  constexpr int QBI = T / 32;        // 16 x 16 blocks per wave, along i
  constexpr int QBJ = T / (16 * WJ);  // and along j
  constexpr int NP = T * BK / (2 * NT);
  __shared__ double As[BK][LS];
  __shared__ double Bs[BK][LS];
  int64_t ti, tj, kbeg, kend;
  int64_t chunk = blockIdx.y;
  int64_t unit = -1;  // split-remainder unit of this workgroup (or -1)
  if (a.gram || a.sym) {
    int64_t t = blockIdx.x;
    if (a.sym && a.nfull >= 0 && t >= a.nfull) {
      unit = t - a.nfull;
      t = a.nfull + unit / a.ksplit;
    }
    ti = 0;
    while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
    tj = t - ti * (ti + 1) / 2;
    kbeg = a.gram ? chunk * a.kchunk : 0;
    kend = a.gram ? min(a.K, kbeg + a.kchunk) : a.K;
    if (unit >= 0) {
      kbeg = (unit % a.ksplit) * a.kpart;
      kend = min(a.K, kbeg + a.kpart);
    }
  } else {
    ti = blockIdx.x;
    tj = blockIdx.y;
    kbeg = 0;
    kend = a.K;
  }
  const int64_t i0 = ti * T, j0 = tj * T;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int qi = (wid / WJ) * (T / 2), qj = (wid % WJ) * (T / WJ);  // block of the wave
  const int li = lane & 15, lk = lane >> 4;
  f64x4 acc[QBI][QBJ];
#pragma unroll
  for (int x = 0; x < QBI; ++x)
#pragma unroll
    for (int y = 0; y < QBJ; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
  // op(B)(k, j) = B(k, j) (tb == 0: contiguous along k) or B(j, k) (tb:
  // contiguous along j): loaded as X(j, k) that is "trans" exactly when tb == 0
  double2 ra[NP], rb[NP];
  if (kbeg < kend) {
    big_load<T, NT, AT>(a.A, a.lda, true, i0, a.M, kbeg, kend, ra);
    big_load<T, NT, BT_>(a.B, a.ldb, a.b_pairs != 0, j0, a.N, kbeg, kend, rb);
  }
  for (int64_t k0 = kbeg; k0 < kend; k0 += BK) {
    __syncthreads();  // the previous slice has been read
    big_store<T, NT, AT>(As, ra, a.dk, k0, kend);
    big_store<T, NT, BT_>(Bs, rb, nullptr, k0, kend);
    __syncthreads();
    if (k0 + BK < kend) {
      big_load<T, NT, AT>(a.A, a.lda, true, i0, a.M, k0 + BK, kend, ra);
      big_load<T, NT, BT_>(a.B, a.ldb, a.b_pairs != 0, j0, a.N, k0 + BK, kend, rb);
    }
    // fragments of step ks + 4 are read from LDS while step ks multiplies
    double fa[2][QBI], fb[2][QBJ];
#pragma unroll
    for (int x = 0; x < QBI; ++x) fa[0][x] = As[lk][qi + 16 * x + li];
#pragma unroll
    for (int y = 0; y < QBJ; ++y) fb[0][y] = Bs[lk][qj + 16 * y + li];
#pragma unroll
    for (int ks = 0; ks < BK; ks += 4) {
      const int cb = (ks / 4) & 1;
      if (ks + 4 < BK) {
#pragma unroll
        for (int x = 0; x < QBI; ++x) fa[cb ^ 1][x] = As[ks + 4 + lk][qi + 16 * x + li];
#pragma unroll
        for (int y = 0; y < QBJ; ++y) fb[cb ^ 1][y] = Bs[ks + 4 + lk][qj + 16 * y + li];
      }
#pragma unroll
      for (int x = 0; x < QBI; ++x)
#pragma unroll
        for (int y = 0; y < QBJ; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[cb][x], fb[cb][y], acc[x][y], 0, 0, 0);
    }
  }
  // accumulator element v of lane l: row 4 v + l / 16, column l % 16 of the block
  if (unit >= 0) {
    double* sp = a.spart + unit * (int64_t)(T * T);
#pragma unroll
    for (int x = 0; x < QBI; ++x)
#pragma unroll
      for (int y = 0; y < QBJ; ++y)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          sp[(qi + 16 * x + 4 * v + lk) + (qj + 16 * y + li) * T] = acc[x][y][v];
    return;
  }
#pragma unroll
  for (int x = 0; x < QBI; ++x)
#pragma unroll
    for (int y = 0; y < QBJ; ++y) {
      const int64_t gj = j0 + qj + 16 * y + li;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t gi = i0 + qi + 16 * x + 4 * v + lk;
        if (gi >= a.M || gj >= a.N) continue;
        if (a.gram) {
          a.part[chunk * a.N * a.N + gi + gj * a.N] = acc[x][y][v];
        } else if (a.sym) {
          if (gi < gj) continue;
          double* cp = a.C + gi + gj * a.ldc;
          const double o = (a.beta == 0.0 ? 0.0 : a.beta * *cp) + a.alpha * acc[x][y][v];
          *cp = o;
          a.C[gj + gi * a.ldc] = o;
        } else if (a.V != nullptr) {
          const double g = (a.gv_p != nullptr) ? *a.gv_p : a.gv;
          const double o = a.alpha * acc[x][y][v];
          a.C[gi + gj * a.ldc] = (g == 0.0) ? o : o + g * a.V[gi + gj * a.ldv];
        } else {
          double* cp = a.C + gi + gj * a.ldc;
          *cp = (a.beta == 0.0 ? 0.0 : a.beta * *cp) + a.alpha * acc[x][y][v];
        }
      }
    }
}

// The split tiles of a symmetric-mode big_gemm_kernel<64, 256> launch, one
// workgroup per tile (tile nfull + blockIdx.x): each entry is the sum of its
// ksplit partial tiles in order of their K parts; the lower entries are
// written as the unsplit kernel writes them, the mirrored ones from an LDS
// copy so that both stores run along columns of C.
__global__ __launch_bounds__(256) void big_sym_split_reduce_kernel(BigGemmArgs a) {
  constexpr int T = 64;
  __shared__ double tile[T][T + 1];
  const int64_t t = a.nfull + blockIdx.x;
  int64_t ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int64_t tj = t - ti * (ti + 1) / 2;
  const double* sp = a.spart + (int64_t)blockIdx.x * a.ksplit * (T * T);
  for (int e = threadIdx.x; e < T * T; e += 256) {
    const int il = e % T, jl = e / T;
    const int64_t gi = ti * T + il, gj = tj * T + jl;
    double o = 0.0;
    if (gi < a.M && gj < a.N && gi >= gj) {
      double sum = 0.0;
      for (int64_t p = 0; p < a.ksplit; ++p) sum += sp[p * (T * T) + e];
      double* cp = a.C + gi + gj * a.ldc;
      o = (a.beta == 0.0 ? 0.0 : a.beta * *cp) + a.alpha * sum;
      *cp = o;
    }
    tile[jl][il] = o;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < T * T; e += 256) {
    const int jl = e % T, il = e / T;
    const int64_t gi = ti * T + il, gj = tj * T + jl;
    if (gi < a.M && gj < a.N && gi > gj) a.C[gj + gi * a.ldc] = tile[jl][il];
  }
}

// Sum of the Gram partials of big_gemm_kernel, one lower tile (ti >= tj) of
// BT x BT per workgroup: the partial tiles are read down their columns
// (coalesced), the sum is written to G as it is and, off the diagonal,
// mirrored through LDS (so that both writes are coalesced too).  The
// chunks are added as four partial sums (chunks c = u mod 4, four loads in
// flight) combined in a fixed order, and a mirrored entry is a copy of its
// lower twin: G is exactly symmetric.
__global__ __launch_bounds__(256) void big_gram_reduce_kernel(int64_t N, int64_t chunks,
                                                              const double* __restrict__ part,
                                                              double* __restrict__ G, int64_t ldg) {
  __shared__ double tile[BT][BT + 1];
  const int64_t t = blockIdx.x;
  int64_t ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int64_t tj = t - ti * (ti + 1) / 2;
  const int64_t i0 = ti * BT, j0 = tj * BT;
  const int r = threadIdx.x % BT, cg = threadIdx.x / BT;
  constexpr int CG = 256 / BT;
  const int64_t NN = N * N;
  const int64_t i = i0 + r;
  for (int cc = cg; cc < BT; cc += CG) {
    const int64_t j = j0 + cc;
    double v = 0.0;
    if (i < N && j < N) {
      const double* p = part + i + j * N;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int64_t c = 0;
      for (; c + 3 < chunks; c += 4) {
        s0 += p[c * NN];
        s1 += p[(c + 1) * NN];
        s2 += p[(c + 2) * NN];
        s3 += p[(c + 3) * NN];
      }
      for (; c < chunks; ++c) s0 += p[c * NN];
      v = (s0 + s1) + (s2 + s3);
      G[i + j * ldg] = v;
    }
    tile[cc][r] = v;
  }
  if (ti == tj) return;  // a diagonal tile holds both triangles of its block
  __syncthreads();
  // G(j0 + r, i0 + cc) = G(i0 + cc, j0 + r), held in tile[r][cc]
  const int64_t jr = j0 + r;
  for (int cc = cg; cc < BT; cc += CG) {
    const int64_t ic = i0 + cc;
    if (jr < N && ic < N) G[jr + ic * ldg] = tile[r][cc];
  }
}

// The same sum, one thread per entry of G (an entry above the diagonal
// tiles reads its lower twin's partials): for Grams of few tiles, whose
// tile-per-workgroup reduction would leave most of the chip idle.
__global__ __launch_bounds__(256) void big_gram_reduce_elem_kernel(int64_t N, int64_t chunks,
                                                                   const double* __restrict__ part,
                                                                   double* __restrict__ G,
                                                                   int64_t ldg) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= N * N) return;
  const int64_t j = e / N, i = e - j * N;
  const bool lower = (i / BT) >= (j / BT);
  const double* p = part + (lower ? (i + j * N) : (j + i * N));
  const int64_t NN = N * N;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t c = 0;
  for (; c + 3 < chunks; c += 4) {
    s0 += p[c * NN];
    s1 += p[(c + 1) * NN];
    s2 += p[(c + 2) * NN];
    s3 += p[(c + 3) * NN];
  }
  for (; c < chunks; ++c) s0 += p[c * NN];
  G[i + j * ldg] = (s0 + s1) + (s2 + s3);
}

// Launch of the Gram reduction: a workgroup per lower tile when there are
// enough tiles to fill the chip, else a thread per entry.
hipError_t launch_big_gram_reduce(int64_t N, int64_t chunks, const double* part, double* G,
                                  int64_t ldg, hipStream_t s) {
  const int64_t T = (N + BT - 1) / BT, tiles = T * (T + 1) / 2;
  if (tiles >= 256)
    hipLaunchKernelGGL(big_gram_reduce_kernel, dim3((unsigned)tiles), dim3(256), 0, s, N, chunks,
                       part, G, ldg);
  else
    hipLaunchKernelGGL(big_gram_reduce_elem_kernel, dim3((unsigned)((N * N + 255) / 256)),
                       dim3(256), 0, s, N, chunks, part, G, ldg);
  return hipGetLastError();
}

// Gram partials over one row chunk for one lower-triangle tile (ti >= tj).
template <typename TP>
__global__ __launch_bounds__(256) void gram_partial_kernel(int64_t d, int64_t N,
                                                           const TP* __restrict__ P, int64_t ldp,
                                                           double* __restrict__ part,
                                                           int64_t rows_per_chunk) {
  __shared__ double As[GK][GT + 1];
  __shared__ double Bs[GK][GT + 1];
  // blockIdx.x enumerates lower-triangle tiles, blockIdx.y row chunks
  int64_t t = blockIdx.x, ti = 0;
  while ((ti + 1) * (ti + 2) / 2 <= t) ++ti;
  const int64_t tj = t - ti * (ti + 1) / 2;
  const int64_t i0 = ti * GT, j0 = tj * GT;
  const int64_t c = blockIdx.y;
  const int64_t r0 = c * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk < d) ? r0 + rows_per_chunk : d;
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  double acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) acc[a][b] = 0.0;

  for (int64_t k0 = r0; k0 < r1; k0 += GK) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + q * 256;
      const int kk = e & 15, ii = e >> 4;
      const int64_t gk = k0 + kk;
      const int64_t gi = i0 + ii, gj = j0 + ii;
      As[kk][ii] = (gi < N && gk < r1) ? to_f64<TP>(P[gk + gi * ldp]) : 0.0;
      Bs[kk][ii] = (gj < N && gk < r1) ? to_f64<TP>(P[gk + gj * ldp]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = As[kk][tx + 16 * q];
#pragma unroll
      for (int q = 0; q < 4; ++q) b[q] = Bs[kk][ty + 16 * q];
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] += a[p] * b[q];
    }
    __syncthreads();
  }
  double* pc = part + c * N * N;
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const int64_t gi = i0 + tx + 16 * p;
    if (gi >= N) continue;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t gj = j0 + ty + 16 * q;
      if (gj >= N) continue;
      pc[gi + gj * N] = acc[p][q];
    }
  }
}

__global__ __launch_bounds__(256) void gram_reduce_kernel(int64_t N, int64_t chunks,
                                                          const double* __restrict__ part,
                                                          double* __restrict__ G, int64_t ldg) {
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= N * N) return;
  const int64_t j = e / N, i = e - j * N;
  // read from the lower-triangle tile that holds (i, j) or its mirror
  const bool lower = (i / GT) >= (j / GT);
  const int64_t src = lower ? (i + j * N) : (j + i * N);
  // four partial sums (chunks c = u mod 4) so that four loads are in
  // flight, added in a fixed order
  const double* p = part + src;
  const int64_t NN = N * N;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int64_t c = 0;
  for (; c + 3 < chunks; c += 4) {
    s0 += p[c * NN];
    s1 += p[(c + 1) * NN];
    s2 += p[(c + 2) * NN];
    s3 += p[(c + 3) * NN];
  }
  for (; c < chunks; ++c) s0 += p[c * NN];
  G[i + j * ldg] = (s0 + s1) + (s2 + s3);
}

void gram_geometry(int64_t d, int64_t N, int64_t* chunks, int64_t* rows) {
  const int64_t T = (N + GT - 1) / GT;
  const int64_t tiles = T * (T + 1) / 2;
  int64_t c = (1024 + tiles - 1) / tiles;
  const int64_t cmax = std::max<int64_t>(1, (d + 255) / 256);
  c = std::max<int64_t>(1, std::min(c, cmax));
  int64_t rp = (d + c - 1) / c;
  rp = ((rp + GK - 1) / GK) * GK;
  *rows = rp;
  *chunks = (d + rp - 1) / rp;
}

// Row chunks of the matrix-core Gram: enough lower-triangle tiles x chunks
// to fill whole rounds of 512 resident workgroups (two per compute unit),
// chunks of at least 256 rows, a multiple of BK.
void big_gram_geometry(int64_t d, int64_t N, int64_t* chunks, int64_t* rows) {
  const int64_t T = (N + BT - 1) / BT;
  const int64_t tiles = T * (T + 1) / 2;
  int64_t best = 1;
  double best_eff = 0.0;
  for (int64_t c = 1; c <= 16; ++c) {
    if (c > 1 && (d + c - 1) / c < 256) break;
    const int64_t wg = tiles * c;
    const int64_t rounds = (wg + 511) / 512;
    const double eff = (double)wg / (double)(rounds * 512);
    if (eff > best_eff + 1e-9) { best_eff = eff; best = c; }
  }
  int64_t rp = (d + best - 1) / best;
  rp = ((rp + BK - 1) / BK) * BK;
  *rows = rp;
  *chunks = (d + rp - 1) / rp;
}

bool big_ok(const double* p, int64_t ld) { return ld % 2 == 0 && ((uintptr_t)p % 16) == 0; }

// big_gemm_kernel<64, 256> instantiated for the operand orientations of a
void launch_big64(dim3 g, hipStream_t s, const BigGemmArgs& a) {
  if (a.ta != 0) {
    if (a.tb != 0)
      hipLaunchKernelGGL((big_gemm_kernel<64, 256, true, false>), g, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((big_gemm_kernel<64, 256, true, true>), g, dim3(256), 0, s, a);
  } else {
    if (a.tb != 0)
      hipLaunchKernelGGL((big_gemm_kernel<64, 256, false, false>), g, dim3(256), 0, s, a);
    else
      hipLaunchKernelGGL((big_gemm_kernel<64, 256, false, true>), g, dim3(256), 0, s, a);
  }
}

// Compute units of the current device (cached per device; 256 if the
// query fails).
int64_t device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cache[dev].load(std::memory_order_relaxed);
  if (v <= 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cache[dev].store(v, std::memory_order_relaxed);
  }
  return v;
}

}  // namespace

hipError_t launch_gemm(bool ta, bool tb, int64_t m, int64_t n, int64_t k, double alpha,
                       const double* A, int64_t lda, const double* dk, const double* B,
                       int64_t ldb, double beta, double* C, int64_t ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (m >= 512 && n >= 512 && k >= 64 && big_ok(A, lda) && big_ok(B, ldb)) {
    BigGemmArgs a{m, n, k, lda, ldb, ldc, A, B, dk, C, alpha, beta, ta ? 1 : 0, tb ? 1 : 0,
                  0, 0, nullptr};
    dim3 g((unsigned)((m + BT - 1) / BT), (unsigned)((n + BT - 1) / BT));
    launch_big64(g, s, a);
    return hipGetLastError();
  }
  dim3 g((unsigned)((m + MT - 1) / MT), (unsigned)((n + MT - 1) / MT));
  hipLaunchKernelGGL(gemm_kernel, g, dim3(256), 0, s, ta, tb, m, n, k, alpha, A, lda, dk, B, ldb,
                     beta, C, ldc);
  return hipGetLastError();
}

hipError_t launch_gemm_av(int64_t m, int64_t n, int64_t k, const double* A, int64_t lda,
                          const double* Z, int64_t ldz, double gv, const double* gv_p,
                          const double* V, int64_t ldv, double* C, int64_t ldc, hipStream_t s) {
  if (m <= 0 || n <= 0) return hipSuccess;
  if (k < BK || !big_ok(A, lda)) return hipErrorInvalidValue;
  BigGemmArgs a{m, n, k, lda, ldz, ldc, A, Z, nullptr, C, 1.0, 0.0, 0, 1, 0, 0, nullptr};
  a.b_pairs = big_ok(Z, ldz) ? 1 : 0;
  a.V = V;
  a.ldv = ldv;
  a.gv = gv;
  a.gv_p = gv_p;
  dim3 g((unsigned)((m + 63) / 64), (unsigned)((n + 63) / 64));
  launch_big64(g, s, a);
  return hipGetLastError();
}

// The matrix-core Gram serves float64 factors with at least 256 columns
// (enough tiles); the register-tiled kernel everything else.
static bool gram_big(int64_t N, DT pdt) { return pdt == DT::F64 && N >= 256; }

// K parts of every tile of a symmetric product of n x n with inner
// dimension k: whole tiles alone leave a compute unit two or three
// workgroups (too few to hide the latency of the slice loop) and a ragged
// last round, so every tile is split along K into ks parts, as many as give
// about eight workgroups a unit (at most 4 parts, at least two slices of BK
// each); 1 when there are tiles enough.
int64_t gemm_sym_split(int64_t n, int64_t k) {
  const int64_t T = (n + 63) / 64, tiles = T * (T + 1) / 2;
  const int64_t cus = device_cus();
  if (n < 512 || k < 64 || tiles >= 8 * cus) return 1;
  int64_t ks = std::min<int64_t>(4, (8 * cus + tiles - 1) / tiles);
  ks = std::min<int64_t>(ks, ((k + BK - 1) / BK) / 2);
  return ks >= 2 ? ks : 1;
}

int64_t gemm_sym_ws_bytes(int64_t n, int64_t k) {
  const int64_t ks = gemm_sym_split(n, k);
  if (ks < 2) return 0;
  const int64_t T = (n + 63) / 64;
  return T * (T + 1) / 2 * ks * 64 * 64 * 8;
}

hipError_t launch_gemm_sym(bool ta, bool tb, int64_t n, int64_t k, double alpha, const double* A,
                           int64_t lda, const double* dk, const double* B, int64_t ldb,
                           double beta, double* C, int64_t ldc, hipStream_t s, double* ws,
                           int64_t ws_bytes) {
  if (n <= 0) return hipSuccess;
  if (n >= 512 && k >= 64 && big_ok(A, lda) && big_ok(B, ldb)) {
    BigGemmArgs a{n, n, k, lda, ldb, ldc, A, B, dk, C, alpha, beta, ta ? 1 : 0, tb ? 1 : 0,
                  0, 0, nullptr};
    a.sym = 1;
    const int64_t T = (n + 63) / 64;
    const int64_t tiles = T * (T + 1) / 2;
    const int64_t ks = gemm_sym_split(n, k);
    if (ks >= 2 && ws != nullptr && ws_bytes >= gemm_sym_ws_bytes(n, k)) {
      const int64_t slices = (k + BK - 1) / BK;
      a.nfull = 0;
      a.ksplit = ks;
      a.kpart = ((slices + ks - 1) / ks) * BK;
      a.spart = ws;
      launch_big64(dim3((unsigned)(tiles * ks)), s, a);
      hipLaunchKernelGGL(big_sym_split_reduce_kernel, dim3((unsigned)tiles), dim3(256), 0, s, a);
      return hipGetLastError();
    }
    launch_big64(dim3((unsigned)tiles), s, a);
    return hipGetLastError();
  }
  return launch_gemm(ta, tb, n, n, k, alpha, A, lda, dk, B, ldb, beta, C, ldc, s);
}

// Gram X^T X of a float64 block of N columns (N >= 48) on the matrix cores:
// lower 64 x 64 tiles x row chunks (about eight workgroups a compute unit,
// at least 512 rows a chunk), partial tiles [chunk][N][N] summed in order
// into G by big_gram_reduce_kernel (mirrored, exactly symmetric).
static void gram_block_geometry(int64_t d, int64_t N, int64_t* chunks, int64_t* rows) {
  const int64_t T = (N + BT - 1) / BT, tiles = T * (T + 1) / 2;
  int64_t c = (8 * device_cus() + tiles - 1) / tiles;
  c = std::max<int64_t>(1, std::min<int64_t>(c, d / 512));
  int64_t rp = (d + c - 1) / c;
  rp = ((rp + BK - 1) / BK) * BK;
  *rows = rp;
  *chunks = (d + rp - 1) / rp;
}

int64_t gram_block_chunks(int64_t d, int64_t N) {
  int64_t c, r;
  gram_block_geometry(d, N, &c, &r);
  return c;
}

hipError_t launch_gram_block(int64_t d, int64_t N, const double* X, int64_t ldx, double* part,
                             int64_t chunks, double* G, int64_t ldg, hipStream_t s) {
  if (d <= 0 || N <= 0) return hipSuccess;
  int64_t c, rows;
  gram_block_geometry(d, N, &c, &rows);
  if (c != chunks || !big_ok(X, ldx)) return hipErrorInvalidValue;
  const int64_t T = (N + BT - 1) / BT;
  BigGemmArgs a{N, N, d, ldx, ldx, N, X, X, nullptr, nullptr, 1.0, 0.0, 1, 0, 1, rows, part};
  launch_big64(dim3((unsigned)(T * (T + 1) / 2), (unsigned)chunks), s, a);
  return launch_big_gram_reduce(N, chunks, part, G, ldg, s);
}

int64_t gram_chunks(int64_t d, int64_t N) {
  int64_t c, r;
  if (gram_big(N, DT::F64))
    big_gram_geometry(d, N, &c, &r);
  else
    gram_geometry(d, N, &c, &r);
  return c;
}

hipError_t launch_gram_partial(int64_t d, int64_t N, const void* P, DT pdt, int64_t ldp,
                               double* part, int64_t chunks, hipStream_t s) {
  int64_t c, rows;
  if (gram_big(N, pdt) && big_ok((const double*)P, ldp)) {
    big_gram_geometry(d, N, &c, &rows);
    if (c != chunks) return hipErrorInvalidValue;
    const int64_t T = (N + BT - 1) / BT;
    BigGemmArgs a{N, N, d, ldp, ldp, N, (const double*)P, (const double*)P, nullptr, nullptr,
                  1.0, 0.0, 1, 0, 1, rows, part};
    launch_big64(dim3((unsigned)(T * (T + 1) / 2), (unsigned)chunks), s, a);
    return hipGetLastError();
  }
  if (gram_big(N, pdt)) return hipErrorInvalidValue;  // chunks were sized for the big kernel
  gram_geometry(d, N, &c, &rows);
  if (c != chunks) return hipErrorInvalidValue;
  const int64_t T = (N + GT - 1) / GT;
  dim3 g((unsigned)(T * (T + 1) / 2), (unsigned)chunks);
  if (pdt == DT::F64)
    hipLaunchKernelGGL(gram_partial_kernel<double>, g, dim3(256), 0, s, d, N, (const double*)P,
                       ldp, part, rows);
  else
    hipLaunchKernelGGL(gram_partial_kernel<float>, g, dim3(256), 0, s, d, N, (const float*)P, ldp,
                       part, rows);
  return hipGetLastError();
}

hipError_t launch_gram_reduce(int64_t N, int64_t chunks, const double* part, double* G,
                              int64_t ldg, hipStream_t s) {
  if (gram_big(N, DT::F64)) {
    return launch_big_gram_reduce(N, chunks, part, G, ldg, s);
  }
  hipLaunchKernelGGL(gram_reduce_kernel, dim3((unsigned)((N * N + 255) / 256)), dim3(256), 0, s, N,
                     chunks, part, G, ldg);
  return hipGetLastError();
}

}  // namespace eda
