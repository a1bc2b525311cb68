// Cholesky factorisation of a small Gram matrix for Cholesky QR:
//   G = W^T W = R^T R,  W <- W R^{-1}.
// One workgroup, the factor kept in LDS (b <= 128).  Outputs R^{-1} in the
// row-major layout read by the nn kernel, and optionally R * Rprev (the
// combined triangular factor of two passes) in column-major order.
//
// Breakdown handling: a pivot that is not positive (the block lost rank in
// floating point) is clamped to a tiny positive value so the division stays
// finite, and *flag is raised; the caller then re-orthogonalises the block.
// With hcol given, *flag is also raised when a column kept less than `ratio`
// of its norm through the preceding projection, the case in which classical
// Gram-Schmidt run twice no longer guarantees orthogonality.
#include "common.h"

namespace eda {

namespace {

constexpr int CH_MAX = 128;

// Orders the LDS accesses of one wave (whose LDS instructions execute in
// program order) without a workgroup barrier.
__device__ __forceinline__ void wave_fence() { __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront"); }

// (largest value, smallest index among equals) over the 64 lanes; the same
// result in every lane
__device__ __forceinline__ void amax_take(double& v, int& i, double ov, int oi) {
  if (ov > v || (ov == v && oi < i)) {
    v = ov;
    i = oi;
  }
}
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int x) {
  return __builtin_amdgcn_update_dpp(0, x, CTRL, 0xF, 0xF, false);
}
__device__ __forceinline__ void wave_argmax(double& v, int& i) {
  amax_take(v, i, dpp_f64<kDppXor1>(v), dpp_i32<kDppXor1>(i));
  amax_take(v, i, dpp_f64<kDppXor2>(v), dpp_i32<kDppXor2>(i));
  amax_take(v, i, dpp_f64<kDppMirror8>(v), dpp_i32<kDppMirror8>(i));
  amax_take(v, i, dpp_f64<kDppMirror16>(v), dpp_i32<kDppMirror16>(i));
  double bv = readlane_f64(v, 0);
  int bi = __builtin_amdgcn_readlane(i, 0);
  for (int row = 16; row < 64; row += 16)
    amax_take(bv, bi, readlane_f64(v, row), __builtin_amdgcn_readlane(i, row));
  v = bv;
  i = bi;
}

// The b x b Gram matrix into LDS (A[r + c*ld], both triangles): copied from
// G, or summed from `chunks` tn partials part[(ch*b + r)*b + c] in chunk
// order.  When b*b is below the thread count, H threads share an entry
// (chunks h, h+H, ...) and their sums are added in order of h through hs
// (blockDim.x doubles).  Ends with a barrier.
__device__ void gram_to_lds(const double* __restrict__ G, int64_t ldg,
                            const double* __restrict__ part, int64_t chunks, int b,
                            double* A, int ld, double* hs) {
  const int nt = blockDim.x, tid = threadIdx.x, bb = b * b;
  if (part == nullptr) {
    for (int e = tid; e < bb; e += nt) {
      const int c = e / b, r = e - c * b;
      A[r + c * ld] = G[r + (int64_t)c * ldg];
    }
    __syncthreads();
    return;
  }
  // H threads per entry, each summing chunks h, h+H, ... in batches of 16
  // loads issued together
  int H = 1;
  while (2 * H * bb <= nt) H *= 2;
  for (int e0 = 0; e0 < bb; e0 += nt / H) {
    const int o = e0 + tid % (nt / H), h = tid / (nt / H);
    double s = 0.0;
    if (o < bb && h < H) {
      const double* p = part + o;
      for (int64_t base = h; base < chunks; base += 16 * (int64_t)H) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int64_t ch = base + (int64_t)u * H;
          v[u] = (ch < chunks) ? p[ch * bb] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; u += 4) s += (v[u] + v[u + 1]) + (v[u + 2] + v[u + 3]);
      }
    }
    if (H > 1) {
      hs[tid] = s;
      __syncthreads();
      if (h == 0 && o < bb) {
        double t = hs[tid];
        for (int q = 1; q < H; ++q) t += hs[q * (nt / H) + tid];
        s = t;
      }
    }
    if (h == 0 && o < bb) {
      const int r = o / b, c = o - r * b;
      A[r + c * ld] = s;
    }
    if (H > 1) __syncthreads();
  }
  __syncthreads();
}

// Cholesky of a symmetric 8 x 8 matrix held by columns in lanes 0..7 of a
// wave (lane c: col[r] = A(r, c)), in registers.  Step j takes the pivot
// from lane j, which scales its column into L(:, j); every lane c > j then
// subtracts L(:, j) L(c, j), reading L(r, j) from lane j.  A pivot not above
// floor_[j] is clamped to it and counted in the return value.  On return
// lane c holds L(r, c) for r >= c, and every lane invd[j] = 1 / L(j, j) and
// pd[j] = the pivot before its square root.
__device__ __forceinline__ int chol8_regs(double (&col)[8], int c, const double (&floor_)[8],
                                          double (&invd)[8], double (&pd)[8]) {
  int bad = 0;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    double djj = readlane_f64(col[j], j);
    pd[j] = djj;
    if (!(djj > floor_[j])) {  // also catches NaN
      djj = floor_[j];
      bad = 1;
    }
    const double piv = sqrt(djj), inv = 1.0 / piv;
    invd[j] = inv;
    const double lcj = col[j] * inv;  // L(c, j) in lane c > j
    if (c == j) {
#pragma unroll
      for (int r = j + 1; r < 8; ++r) col[r] *= inv;
      col[j] = piv;
    }
#pragma unroll
    for (int r = j + 1; r < 8; ++r) {
      const double lrj = readlane_f64(col[r], j);
      if (c > j) col[r] -= lrj * lcj;
    }
  }
  return bad;
}

// Column c of L^{-1} (forward substitution on e_c) from the output of
// chol8_regs; lane c gets y[r] = (L^{-1})(r, c), so (L^{-T})(c, q) = y[q]
// is row c of R^{-1} for R = L^T.
__device__ __forceinline__ void inv8_regs(const double (&col)[8], int c, const double (&invd)[8],
                                          double (&y)[8]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    double sacc = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int k = 0; k < r; ++k) sacc -= readlane_f64(col[r], k) * y[k];
    y[r] = sacc * invd[r];
  }
}

// The inputs of a narrow block (b <= 16) with one memory round trip: every
// thread issues all of its global loads (the gate, Rprev, the projection
// coefficients, the Gram entries or their chunk partials) before it uses
// any of them, then one barrier.  Results: A[r + c*ld] the Gram matrix (sums
// in the order of gram_to_lds), hn[c] = sum_r hcol[r, c]^2 when hcol is
// given (rows in a fixed order), RP[r + c*64] = Rprev when RP is given.
// hs, hs2: blockDim.x doubles each.  Returns the gate's value (1 without a
// gate); the buffers behind a closed gate are still valid, only stale.
__device__ int stage_small(const double* __restrict__ G, int64_t ldg,
                           const double* __restrict__ part, int64_t chunks, int b, double* A,
                           int ld, double* hs, double* hs2, const double* __restrict__ hcol,
                           int64_t m, int64_t ldhc, double* hn, const double* __restrict__ Rprev,
                           int64_t ldrp, double* RP, const int* gate) {
  const int nt = blockDim.x, tid = threadIdx.x, bb = b * b;
  const int gv = (gate != nullptr) ? *gate : 1;
  double rp = 0.0;
  if (RP != nullptr && tid < bb) rp = Rprev[(tid % b) + (int64_t)(tid / b) * ldrp];
  // projection coefficients: column tid % b, rows tid / b + k * per
  const int per = nt / b;
  double h2 = 0.0;
  if (hcol != nullptr && tid < per * b) {
    const double* hc = hcol + (int64_t)(tid % b) * ldhc;
    for (int64_t r = tid / b; r < m; r += 8 * (int64_t)per) {
      double v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int64_t rr = r + (int64_t)u * per;
        v[u] = (rr < m) ? hc[rr] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) h2 += v[u] * v[u];
    }
  }
  // Gram entry o by H threads (chunks h, h+H, ...), as in gram_to_lds
  int H = 1;
  if (part != nullptr)
    while (2 * H * bb <= nt) H *= 2;
  const int st = nt / H;
  const int o = tid % st, h = tid / st;
  double g = 0.0;
  if (o < bb && h < H) {
    if (part == nullptr) {
      g = G[(o % b) + (int64_t)(o / b) * ldg];
    } else {
      const double* p = part + o;
      for (int64_t base = h; base < chunks; base += 16 * (int64_t)H) {
        double v[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int64_t ch = base + (int64_t)u * H;
          v[u] = (ch < chunks) ? p[ch * bb] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; u += 4) g += (v[u] + v[u + 1]) + (v[u + 2] + v[u + 3]);
      }
    }
  }
  hs[tid] = g;
  hs2[tid] = h2;
  if (RP != nullptr && tid < bb) RP[(tid % b) + (tid / b) * 64] = rp;
  __syncthreads();
  if (tid < bb) {
    double t = hs[tid];
    if (part != nullptr) {
      // entry tid: partial sums of threads tid + q st, q = 0..H-1, in order
      for (int q = 1; q < H; ++q) t += hs[q * st + tid];
      const int r = tid / b, c = tid - r * b;  // partials are row-major
      A[r + c * ld] = t;
    } else {
      A[(tid % b) + (tid / b) * ld] = t;  // G is column-major
    }
  }
  if (hcol != nullptr && tid < b) {
    double t = 0.0;
    for (int q = 0; q < per; ++q) t += hs2[tid + q * b];
    hn[tid] = t;
  }
  __syncthreads();
  return gv;
}

// LDS use of chol_kernel (one b x b array, ld = CH_MAX + 1): the Gram
// matrix, then L in its lower triangle (diagonal also in rd); for b > 8 the
// columns of L^{-1} go to the strict upper triangle (L^{-1}(r, c) at (c, r)),
// their diagonal to xd.  Rprev (b <= 64) is staged in columns 64.. .
__global__ __launch_bounds__(256) void chol_kernel(const CholArgs* __restrict__ arr, CholArgs one) {
  const CholArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int b = (int)a.b;
  const double* __restrict__ G = a.G;
  double* __restrict__ Rinv = a.Rinv;
  const double* __restrict__ Rprev = a.Rprev;
  double* __restrict__ Rout = a.Rout;
  const double* __restrict__ hcol = a.hcol;
  const int64_t ldg = a.ldg, ldri = a.ldri, ldrp = a.ldrp, ldro = a.ldro, m = a.m, ldhc = a.ldhc;
  const double ratio = a.ratio;
  int* flag = a.flag;
  __shared__ double L[CH_MAX * (CH_MAX + 1)];
  __shared__ double rd[CH_MAX], xd[CH_MAX], hn[CH_MAX], d0[CH_MAX], hs[256], hs2[256];
  __shared__ int sflag;
  const int ld = CH_MAX + 1;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6, nw = blockDim.x >> 6;
  if (tid == 0) sflag = 0;
  // Rprev (b <= 64) staged in the unused second half of L
  double* RP = (Rprev != nullptr && b <= 64) ? L + 64 * ld : nullptr;
  if (b <= 16) {
    // narrow blocks: every input in one memory round trip, the gate included
    if (stage_small(G, ldg, a.part, a.chunks, b, L, ld, hs, hs2, hcol, m, ldhc, hn, Rprev, ldrp,
                    RP, a.gate) == 0)
      return;
  } else {
    if (a.gate != nullptr && *a.gate == 0) return;
    if (RP != nullptr)
      for (int e = tid; e < b * b; e += blockDim.x) {
        const int c = e / b, r = e - c * b;
        RP[r + c * 64] = Rprev[r + c * ldrp];
      }
    gram_to_lds(G, ldg, a.part, a.chunks, b, L, ld, hs);
    // squared norms of the projection coefficients, one wave per column
    if (hcol != nullptr)
      for (int c = wid; c < b; c += nw) {
        const double* hc = hcol + (int64_t)c * ldhc;
        const double v0 = (lane < m) ? hc[lane] : 0.0;
        const double v1 = (lane + 64 < m) ? hc[lane + 64] : 0.0;
        double h2 = v0 * v0 + v1 * v1;
        for (int64_t r = lane + 128; r < m; r += 64) h2 += hc[r] * hc[r];
        h2 = wave_sum(h2);
        if (lane == 0) hn[c] = h2;
      }
  }
  for (int r = tid; r < b; r += blockDim.x) d0[r] = L[r + r * ld];
  __syncthreads();
  if (b <= 8) {
    // Blocks of at most 8 columns: wave 0 factorises and inverts in
    // registers (the matrix identity-padded to 8; only its lower triangle is
    // read, so the copy in registers is exactly symmetric).
    if (wid == 0) {
      const int c = lane;
      double col[8], fl[8], invd[8], pd[8], y[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const bool in = c < b && r < b;
        const double g = in ? ((r >= c) ? L[r + c * ld] : L[c + r * ld]) : 0.0;
        col[r] = in ? g : ((r == c) ? 1.0 : 0.0);
        fl[r] = (r < b) ? 1e-28 * fabs(d0[r]) + 1e-300 : 0.0;
      }
      int bad = chol8_regs(col, c, fl, invd, pd);
      inv8_regs(col, c, invd, y);
      if (Rout != nullptr) {
        // lane q: column q of R Rprev (or of R), R(i, k) = L(k, i):
        //   (R Rprev)(i, q) = sum_{k >= i} L(k, i) Rprev(k, q)
        double rq[8], o[8];
#pragma unroll
        for (int k = 0; k < 8; ++k)
          rq[k] = (Rprev != nullptr) ? ((c < b && k < b) ? RP[k + c * 64] : 0.0)
                                     : ((k == c) ? 1.0 : 0.0);
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          double sacc = 0.0;
#pragma unroll
          for (int k = i; k < 8; ++k) sacc += readlane_f64(col[k], i) * rq[k];
          o[i] = sacc;
        }
        if (c < b)
#pragma unroll
          for (int i = 0; i < 8; ++i)
            if (i < b) Rout[i + (int64_t)c * ldro] = o[i];
      }
      if (c < b) {
        // row c of R^{-1} (row-major)
#pragma unroll
        for (int q = 0; q < 8; ++q)
          if (q < b) Rinv[(int64_t)c * ldri + q] = y[q];
        if (hcol != nullptr) {
          double rc = 0.0;
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (k == c) rc = col[k];
          if (!(rc >= ratio * sqrt(hn[c] + rc * rc))) bad = 1;
        }
      }
      if (bad && c < 8) sflag = 1;
    }
    __syncthreads();
    if (tid == 0 && flag != nullptr && sflag) *flag = 1;
    return;
  }
  // A Gram matrix within 1e-10 of the identity (the second pass of Cholesky
  // QR): with E = G - I, R = I + F + O(|E|^2) where F is the strict upper
  // triangle of E plus half its diagonal, and R^{-1} = I - F + O(|E|^2); the
  // neglected terms are below b 1e-20.  (NaN fails the test.)
  if (Rprev == nullptr && hcol == nullptr) {
    int far = 0;
    for (int e = tid; e < b * b; e += blockDim.x) {
      const int c = e / b, r = e - c * b;
      if (r >= c && !(fabs(L[r + c * ld] - (r == c ? 1.0 : 0.0)) <= 1e-10)) far = 1;
    }
    if (__syncthreads_or(far) == 0) {
      for (int e = tid; e < b * b; e += blockDim.x) {
        const int i = e / b, c = e - i * b;  // R^{-1}(i, c), row-major; E(i, c) = L(c, i), i < c
        Rinv[(int64_t)i * ldri + c] =
            (c > i) ? -L[c + i * ld] : (c == i ? 1.0 - 0.5 * (L[i + i * ld] - 1.0) : 0.0);
      }
      if (Rout != nullptr)
        for (int e = tid; e < b * b; e += blockDim.x) {
          const int c = e / b, r = e - c * b;
          Rout[r + (int64_t)c * ldro] =
              (r < c) ? L[c + r * ld] : (r == c ? 1.0 + 0.5 * (L[r + r * ld] - 1.0) : 0.0);
        }
      return;
    }
  }
  // Wider blocks (8 < b <= 128): blocked right-looking factorisation with 8 x 8
  // diagonal blocks, three barriers per block column.  Per block column
  // kb: wave 0 factorises and inverts the diagonal block in registers (as
  // above); every thread then takes rows of the panel below,
  // L21 = A21 L11^{-T}; then the threads update the trailing lower
  // triangle, A22 -= L21 L21^T.  L stays in the lower triangle of the LDS
  // array, rd holds its diagonal.
  __shared__ double Lis[CH_MAX / 8][64];  // L11^{-1} of every diagonal block, [kb][r * 8 + c]
  const int nblk = (b + 7) / 8;
  for (int kb = 0; kb < nblk; ++kb) {
    const int k0 = 8 * kb, kw = (b - k0 < 8) ? b - k0 : 8;
    if (wid == 0) {
      const int c = lane;
      double col[8], fl[8], invd[8], pd[8], y[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const bool in = c < kw && r < kw;
        const double g = in ? ((r >= c) ? L[(k0 + r) + (k0 + c) * ld] : L[(k0 + c) + (k0 + r) * ld])
                            : 0.0;
        col[r] = in ? g : ((r == c) ? 1.0 : 0.0);
        fl[r] = (r < kw) ? 1e-28 * fabs(d0[k0 + r]) + 1e-300 : 0.0;
      }
      const int bad = chol8_regs(col, c, fl, invd, pd);
      inv8_regs(col, c, invd, y);
      if (c < kw) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          if (r >= c && r < kw) L[(k0 + r) + (k0 + c) * ld] = col[r];
          if (r == c) rd[k0 + c] = col[r];
          Lis[kb][r * 8 + c] = y[r];
        }
      }
      if (bad && c < 8) sflag = 1;
    }
    __syncthreads();
    const int p0 = k0 + kw;
    // panel: L21[i][c] = sum_{q <= c} A21[i][q] (L11^{-1})[c][q]
    for (int i = p0 + tid; i < b; i += blockDim.x) {
      double av[8], o[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) av[q] = (q < kw) ? L[i + (k0 + q) * ld] : 0.0;
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        double sacc = 0.0;
#pragma unroll
        for (int q = 0; q <= c; ++q) sacc += av[q] * Lis[kb][c * 8 + q];
        o[c] = sacc;
      }
#pragma unroll
      for (int c = 0; c < 8; ++c)
        if (c < kw) L[i + (k0 + c) * ld] = o[c];
    }
    __syncthreads();
    // trailing lower triangle: A22 -= L21 L21^T
    const int rem = b - p0;
    for (int e = tid; e < rem * rem; e += blockDim.x) {
      const int cc = e / rem, rr = e - cc * rem;
      if (rr < cc) continue;
      const int r = p0 + rr, c = p0 + cc;
      double sacc = 0.0;
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q < kw) sacc += L[r + (k0 + q) * ld] * L[c + (k0 + q) * ld];
      L[r + c * ld] -= sacc;
    }
    __syncthreads();
  }
  // Y = L^{-1} by block rows I (rows r0 .. r0+kw-1), two barriers each:
  //   T(r, c) = sum_{k=c}^{r0-1} L(r, k) Y(k, c)  for c < r0 (earlier block rows final),
  //   Y(r, c) = -(L_II^{-1} T)(r, c),   Y_II = L_II^{-1}.
  // Y(r, c), r > c, goes to the upper position (c, r), its diagonal to xd;
  // then R^{-1} = Y^T: row i of R^{-1} is column i of Y.
  __shared__ double Tb[8 * CH_MAX];
  for (int I = 0; I < nblk; ++I) {
    const int r0 = 8 * I, kw = (b - r0 < 8) ? b - r0 : 8;
    for (int e = tid; e < kw * r0; e += blockDim.x) {
      const int c = e / kw, j = e - c * kw;
      // four independent partial sums (LDS loads of four k in flight), added
      // in a fixed order
      const double* lr = L + (r0 + j);
      double s0 = lr[c * ld] * xd[c], s1 = 0.0, s2 = 0.0, s3 = 0.0;
      int k = c + 1;
      for (; k + 3 < r0; k += 4) {
        s0 += lr[k * ld] * L[c + k * ld];
        s1 += lr[(k + 1) * ld] * L[c + (k + 1) * ld];
        s2 += lr[(k + 2) * ld] * L[c + (k + 2) * ld];
        s3 += lr[(k + 3) * ld] * L[c + (k + 3) * ld];
      }
      for (; k < r0; ++k) s0 += lr[k * ld] * L[c + k * ld];
      Tb[j * CH_MAX + c] = (s0 + s1) + (s2 + s3);
    }
    __syncthreads();
    for (int e = tid; e < kw * r0; e += blockDim.x) {
      const int c = e / kw, j = e - c * kw;
      double sacc = 0.0;
      for (int q = 0; q <= j; ++q) sacc += Lis[I][j * 8 + q] * Tb[q * CH_MAX + c];
      L[c + (r0 + j) * ld] = -sacc;
    }
    for (int e = tid; e < kw * kw; e += blockDim.x) {
      const int j = e / kw, q = e - j * kw;
      if (q < j)
        L[(r0 + q) + (r0 + j) * ld] = Lis[I][j * 8 + q];
      else if (q == j)
        xd[r0 + j] = Lis[I][j * 8 + j];
    }
    __syncthreads();
  }
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int i = e / b, c = e - i * b;  // R^{-1}(i, c) = Y(c, i), zero for c < i
    Rinv[(int64_t)i * ldri + c] = (c > i) ? L[i + c * ld] : (c == i ? xd[i] : 0.0);
  }
  if (Rout != nullptr) {
    for (int e = tid; e < b * b; e += blockDim.x) {
      const int c = e / b, r = e - c * b;
      // R(r, q) = L(q, r) for q >= r; (R Rprev)(r, c) = sum_{q >= r} R(r, q) Rprev(q, c)
      double sacc = 0.0;
      if (Rprev == nullptr) {
        sacc = (r < c) ? L[c + r * ld] : (r == c ? rd[r] : 0.0);
      } else if (RP != nullptr) {
        sacc = rd[r] * RP[r + c * 64];
        for (int q = r + 1; q < b; ++q) sacc += L[q + r * ld] * RP[q + c * 64];
      } else {
        sacc = rd[r] * Rprev[r + c * ldrp];
        for (int q = r + 1; q < b; ++q) sacc += L[q + r * ld] * Rprev[q + c * ldrp];
      }
      Rout[r + c * ldro] = sacc;
    }
  }
  if (hcol != nullptr && tid < b) {
    const double rc = rd[tid];
    if (!(rc >= ratio * sqrt(hn[tid] + rc * rc))) atomicOr(&sflag, 1);
  }
  __syncthreads();
  if (tid == 0 && flag != nullptr && sflag) *flag = 1;
}

// Rank-revealing (diagonally pivoted) Cholesky of a Lanczos block's Gram
// matrix G = W^T W, b <= 64, W already projected against the basis with
// coefficients hcol (m x b).  Columns whose remaining pivot is below
// (tau * scale)^2, scale^2 = max_j (||h_j||^2 + G_jj) being the largest
// squared column norm before the projection, are deflated: the Krylov space
// has become invariant along them.  With r kept columns and permutation p:
//   W P = [Q_1 Q_2] [[R11 R12], [0, ~0]],   Q_1 = W P[:, :r] R11^{-1}.
// Outputs: Z (row-major, W Z = [Q_1, 0]), R (col-major, W = [Q_1 Q_2] R with
// rows >= r zero), mask[j] = 1 for deflated output columns j >= r, and
// *flag = 1 if a column kept less than `ratio` of its norm, | 2 if a column
// was deflated (nothing is written when neither happened).
__global__ __launch_bounds__(256) void pchol_kernel(const PcholArgs* __restrict__ arr, PcholArgs one) {
  const PcholArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int b = (int)a.b;
  const double* __restrict__ G = a.G;
  const double* __restrict__ hcol = a.hcol;
  const int64_t ldg = a.ldg, m = a.m, ldhc = a.ldhc, ldz = a.ldz, ldr = a.ldr;
  const double tau = a.tau, ratio = a.ratio;
  const int equil = a.equil;
  double* __restrict__ Z = a.Z;
  double* __restrict__ R = a.R;
  int* __restrict__ mask = a.mask;
  int* flag = a.flag;
  constexpr int PB = 64;
  __shared__ double A[PB * (PB + 1)];
  __shared__ double nrm0[PB];
  __shared__ double dsc[PB];  // column scaling (1 unless equilibrated)
  __shared__ int perm[PB];
  __shared__ int s_rank, s_flag;
  __shared__ double gd[PB], hs[256], hs2[256], hn[PB];
  const int ld = PB + 1;
  const int tid = threadIdx.x;
  const bool narrow = b <= 16;  // then every input arrives in one memory round trip
  if (narrow)
    stage_small(G, ldg, a.part, a.chunks, b, A, ld, hs, hs2, equil ? nullptr : hcol, m, ldhc, hn,
                nullptr, 0, nullptr, nullptr);
  else
    gram_to_lds(G, ldg, a.part, a.chunks, b, A, ld, hs);
  if (a.corr != nullptr) {
    // G -= corr^T corr: the Gram matrix of W - Q h from that of W and the
    // coefficients h = Q^T W (Q orthonormal, h row-major mcorr x b); h is
    // staged in tiles of 2048 / b rows, one memory round trip per tile
    __shared__ double cs[2048];
    const int64_t kt = 2048 / b;
    for (int64_t k0 = 0; k0 < a.mcorr; k0 += kt) {
      const int64_t kn = (a.mcorr - k0 < kt) ? a.mcorr - k0 : kt;
      __syncthreads();  // the previous tile has been read
      for (int64_t e = tid; e < kn * b; e += blockDim.x) cs[e] = a.corr[k0 * b + e];
      __syncthreads();
      for (int e = tid; e < b * b; e += blockDim.x) {
        const int c = e / b, r = e - c * b;
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        int64_t k = 0;
        for (; k + 4 <= kn; k += 4)
#pragma unroll
          for (int u = 0; u < 4; ++u) acc[u] = fma(cs[(k + u) * b + r], cs[(k + u) * b + c], acc[u]);
        for (; k < kn; ++k) acc[0] = fma(cs[k * b + r], cs[k * b + c], acc[0]);
        A[r + c * ld] -= (acc[0] + acc[1]) + (acc[2] + acc[3]);
      }
    }
    __syncthreads();
  }
  if (tid < b) {
    const double g = A[tid + tid * ld];
    gd[tid] = g;
    dsc[tid] = (equil && g > 0.0) ? 1.0 / sqrt(g) : 1.0;
  }
  __syncthreads();
  if (equil)
    for (int e = tid; e < b * b; e += blockDim.x) {
      const int c = e / b, r = e - c * b;
      A[r + c * ld] *= dsc[r] * dsc[c];
    }
  // squared norms of the projection coefficients: the wave sums column c
  // and lane c keeps it
  double h2 = 0.0;
  if (hcol != nullptr && !equil && narrow) {
    if (tid < b) h2 = hn[tid];
  } else if (hcol != nullptr && !equil)
    for (int c0 = 0; c0 < b; c0 += 8) {
      double hs[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double* hc = hcol + (int64_t)(c0 + u < b ? c0 + u : 0) * ldhc;
        const double v0 = (c0 + u < b && tid < m) ? hc[tid] : 0.0;
        const double v1 = (c0 + u < b && tid + 64 < m) ? hc[tid + 64] : 0.0;
        hs[u] = v0 * v0 + v1 * v1;
        if (c0 + u < b)
          for (int64_t r = tid + 128; r < m; r += 64) hs[u] += hc[r] * hc[r];
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const double t = wave_sum(hs[u]);
        if (tid == c0 + u) h2 = t;
      }
    }
  if (tid < b) {
    nrm0[tid] = gd[tid] * dsc[tid] * dsc[tid] + h2;
    perm[tid] = tid;
  }
  if (tid == 0) {
    s_rank = b;
    s_flag = 0;
  }
  __syncthreads();
  double scale2 = 0.0;
  for (int j = 0; j < b; ++j) scale2 = fmax(scale2, nrm0[j]);
  const double thr = tau * tau * scale2;
  if (b <= 8) {
    // First the unpivoted factorisation in registers (as in chol_kernel).
    // When every pivot keeps at least 1e-8 of its column's squared norm in
    // the block (and is far above the deflation threshold), no column is
    // near the span of the others and the identity is as good a pivot order
    // as any: its outputs are final.  Otherwise the pivoted factorisation
    // below runs on the untouched LDS copy.
    __shared__ int s_fast;
    if (tid < 64) {
      const int c = tid;
      double col[8], fl[8], invd[8], pd[8], y[8], g0[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const bool in = c < b && r < b;
        const double g = in ? ((r >= c) ? A[r + c * ld] : A[c + r * ld]) : 0.0;
        col[r] = in ? g : ((r == c) ? 1.0 : 0.0);
        fl[r] = 0.0;
      }
#pragma unroll
      for (int r = 0; r < 8; ++r) g0[r] = readlane_f64(col[r], r);
      int bad = chol8_regs(col, c, fl, invd, pd);
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (j < b && !(pd[j] > fmax(1e-8 * g0[j], 1e6 * thr))) bad = 1;
      if (!bad) {
        inv8_regs(col, c, invd, y);
        if (c < b) {
          const double sc = dsc[c];
          // row c of Z = R^{-1} (times the column scaling when equilibrated)
#pragma unroll
          for (int q = 0; q < 8; ++q)
            if (q < b) Z[(int64_t)c * ldz + q] = equil ? y[q] * sc : y[q];
          // row c of R: R(c, k) = L(k, c) / dsc[k] for k >= c
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (k < b) R[c + (int64_t)k * ldr] = (k >= c) ? col[k] / dsc[k] : 0.0;
          mask[c] = 0;
          double rc = 0.0;
#pragma unroll
          for (int k = 0; k < 8; ++k)
            if (k == c) rc = col[k];
          if (!(rc >= ratio * sqrt(nrm0[c]))) s_flag = 1;
        }
      }
      if (c == 0) s_fast = !bad;
    }
    __syncthreads();
    if (s_fast) {
      if (tid == 0 && flag != nullptr && s_flag) *flag = 1;
      return;
    }
  }
  // The factorisation runs in wave 0 alone (b <= 64: lane r owns row and
  // column r), so its steps need no workgroup barrier.
  if (tid < 64) {
    const int r = tid;
    const bool live = r < b;
    int pr = r;  // perm entry of position r
    int rank = b;
    for (int j = 0; j < b; ++j) {
      double v = (live && r >= j) ? A[r + r * ld] : -INFINITY;
      int vi = r;
      wave_argmax(v, vi);
      if (!(v > thr)) {  // every remaining pivot is negligible: deflate them
        rank = j;
        break;
      }
      const int q = vi;
      if (q != j) {
        const int pj = __builtin_amdgcn_readlane(pr, j), pq = __builtin_amdgcn_readlane(pr, q);
        if (r == j) pr = pq;
        if (r == q) pr = pj;
        if (live) {  // swap rows j and q
          const double t = A[j + r * ld];
          A[j + r * ld] = A[q + r * ld];
          A[q + r * ld] = t;
        }
        wave_fence();
        if (live) {  // swap columns j and q
          const double t = A[r + j * ld];
          A[r + j * ld] = A[r + q * ld];
          A[r + q * ld] = t;
        }
        wave_fence();
      }
      const double piv = sqrt(A[j + j * ld]);
      const double lr = (live && r > j) ? A[r + j * ld] / piv : 0.0;
      wave_fence();
      if (r == j) A[j + j * ld] = piv;
      if (live && r > j) A[r + j * ld] = lr;
      // update the whole (symmetric) trailing block: later pivot swaps read
      // both of its triangles
      for (int c = j + 1; c < b; ++c) {
        const double lc = readlane_f64(lr, c);
        if (live && r > j) A[r + c * ld] -= lr * lc;
      }
      wave_fence();
    }
    if (live) perm[r] = pr;
    if (r == 0) s_rank = rank;
  }
  __syncthreads();
  const int rk = s_rank;
  __shared__ double xd[PB];
  __shared__ int iperm[PB];
  if (tid < b) iperm[perm[tid]] = tid;
  // R11^{-1} (upper, R11[i][q] = L[q][i]) by back substitution, one thread
  // per column c < rk; X[i][c] (i < c) goes to the strict upper triangle of
  // A, which the factorisation no longer needs, the diagonal to xd.
  if (tid < rk) {
    const int c = tid;
    const double xcc = 1.0 / A[c + c * ld];
    xd[c] = xcc;
    for (int i = c - 1; i >= 0; --i) {
      double s = -A[c + i * ld] * xcc;
      for (int q = i + 1; q < c; ++q) s -= A[q + i * ld] * A[q + c * ld];
      A[i + c * ld] = s / A[i + i * ld];
    }
  }
  __syncthreads();
  // Z[rho][c] = X[i][c] with perm[i] = rho (zero for i > c or c >= rk),
  // times the column scaling of rho when equilibrated
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int rho = e / b, c = e - rho * b;
    const int i = iperm[rho];
    double v = 0.0;
    if (c < rk && i <= c) v = (i < c) ? A[i + c * ld] : xd[c];
    Z[(int64_t)rho * ldz + c] = equil ? v * dsc[rho] : v;
  }
  // R[j, perm[i]] = L[i, j] for j < rk, i >= j; zero elsewhere.
  for (int e = tid; e < b * b; e += blockDim.x) {
    const int ci = e / b, j = e - ci * b;  // output column ci (original index), row j
    const int i = iperm[ci];
    const double v = (j < rk && i >= j) ? A[i + j * ld] / dsc[ci] : 0.0;
    R[j + (int64_t)ci * ldr] = v;
  }
  if (tid < b) {
    mask[tid] = (tid >= rk) ? 1 : 0;
    if (tid < rk && !(A[tid + tid * ld] >= ratio * sqrt(nrm0[perm[tid]]))) atomicOr(&s_flag, 1);
  }
  __syncthreads();
  if (tid == 0 && flag != nullptr && (s_flag || rk < b)) *flag = (s_flag ? 1 : 0) | (rk < b ? 2 : 0);
}

// Q[:, j] = seeded Gaussian for every column j with mask[j] != 0.
template <typename T>
__global__ __launch_bounds__(256) void fill_masked_randn_kernel(const MaskedRandnArgs* __restrict__ arr,
                                                                MaskedRandnArgs one) {
  const MaskedRandnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  const int64_t d = a.d, b = a.b, ldq = a.ldq;
  const int* __restrict__ mask = a.mask;
  const uint64_t seed = a.seed;
  T* Q = (T*)a.Q;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (e >= d * b) return;
  const int64_t c = e / d, r = e - c * d;
  if (mask[c] == 0) return;
  Q[r + c * ldq] = from_f64<T>(masked_gauss(seed, e));
}

}  // namespace

hipError_t launch_pchol_multi(int count, const PcholArgs* host, const PcholArgs* dev,
                              hipStream_t s) {
  if (count < 1) return hipSuccess;
  for (int p = 0; p < count; ++p)
    if (host[p].b < 1 || host[p].b > 64) return hipErrorInvalidValue;
  const PcholArgs* arr;
  PcholArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(pchol_kernel, dim3(1, 1, (unsigned)count), dim3(256), 0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_pchol(int64_t b, const double* G, int64_t ldg, const double* hcol, int64_t m,
                        int64_t ldhc, double tau, double ratio, bool equil, double* Z, int64_t ldz,
                        double* R, int64_t ldr, int* mask, int* flag, hipStream_t s,
                        const double* part, int64_t chunks, const double* corr, int64_t mcorr) {
  if (corr != nullptr && mcorr < 0) return hipErrorInvalidValue;
  PcholArgs a{b, ldg, m, ldhc, ldz, ldr, G, hcol, tau, ratio, equil ? 1 : 0, Z, R, mask, flag,
              part, chunks};
  a.corr = corr;
  a.mcorr = mcorr;
  return launch_pchol_multi(1, &a, nullptr, s);
}

hipError_t launch_masked_randn_multi(int count, const MaskedRandnArgs* host,
                                     const MaskedRandnArgs* dev, DT qdt, hipStream_t s) {
  int64_t x = 0;
  for (int p = 0; p < count; ++p) x = std::max<int64_t>(x, (host[p].d * host[p].b + 255) / 256);
  if (x == 0) return hipSuccess;
  const MaskedRandnArgs* arr;
  MaskedRandnArgs one;
  pick(count, host, dev, &arr, &one);
  const dim3 g((unsigned)x, 1, (unsigned)count);
  if (qdt == DT::F64)
    hipLaunchKernelGGL(fill_masked_randn_kernel<double>, g, dim3(256), 0, s, arr, one);
  else if (qdt == DT::F32)
    hipLaunchKernelGGL(fill_masked_randn_kernel<float>, g, dim3(256), 0, s, arr, one);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_fill_masked_randn(int64_t d, int64_t b, const int* mask, uint64_t seed,
                                    void* Q, DT qdt, int64_t ldq, hipStream_t s) {
  MaskedRandnArgs a{d, b, ldq, mask, seed, Q};
  return launch_masked_randn_multi(1, &a, nullptr, qdt, s);
}

hipError_t launch_chol_multi(int count, const CholArgs* host, const CholArgs* dev, hipStream_t s) {
  if (count < 1) return hipSuccess;
  for (int p = 0; p < count; ++p)
    if (host[p].b < 1 || host[p].b > CH_MAX) return hipErrorInvalidValue;
  const CholArgs* arr;
  CholArgs one;
  pick(count, host, dev, &arr, &one);
  hipLaunchKernelGGL(chol_kernel, dim3(1, 1, (unsigned)count), dim3(256), 0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_chol(int64_t b, const double* G, int64_t ldg, double* Rinv, int64_t ldri,
                       const double* Rprev, int64_t ldrp, double* Rout, int64_t ldro,
                       const double* hcol, int64_t m, int64_t ldhc, double ratio, int* flag,
                       const int* gate, hipStream_t s, const double* part, int64_t chunks) {
  CholArgs a{b, ldg, ldri, ldrp, ldro, m, ldhc, G, Rinv, Rprev, Rout, hcol, ratio, flag, gate,
             part, chunks};
  return launch_chol_multi(1, &a, nullptr, s);
}

}  // namespace eda
