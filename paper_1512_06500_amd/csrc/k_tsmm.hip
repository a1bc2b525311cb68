// Tall-skinny products that stream a d x m matrix once from HBM.
//
//   tn:  part[c] = A[rows_c, :]^T B[rows_c, :]   (A: d x m, B: d x nb, nb small)
//        followed by a fixed-order sum over the row chunks c (deterministic).
//   nn:  Out = alpha V + A Z                    (A: d x m, Z: m x nb)
//
// These are the two passes of the low-rank exponential apply
//   exp(c H H^T) V = V + H G_c (H^T V)
// (Theorem 3.1 in Gram form) and also the projections of block classical
// Gram-Schmidt and the W R^{-1} step of Cholesky QR.  Both are HBM-bound:
// for nb = 8 every element of A feeds 8 FMAs, far below the FP64 ridge, so
// the design goal is to keep enough loads in flight, never to save flops.
//
// tn mapping: the row reduction is done by the matrix cores.  One
// v_mfma_f64_16x16x4f64 takes a 16 x 4 slice of A^T and a 4 x 16 slice of B
// and accumulates their product, so a wave owns 16 columns of A (and up to
// 16 of B) and sums over 4 rows per instruction without any cross-lane
// shuffles.  Lane (i = l % 16, q = l / 16) reads 16 consecutive rows of
// column i (and of B's column i), i.e. every cache line fetched is consumed
// by the same lane over 16 instructions; which k slot a row occupies does
// not matter for a sum.  The 4 waves of a workgroup take 4 consecutive
// 64 S-row ranges of one 16-column tile and are summed through LDS, so each
// workgroup writes one partial tile.
//
// nn mapping: a workgroup owns R rows and all m columns; its 256 lanes are
// R rows x G = 256/R column groups (column j goes to group j mod G), so every
// lane issues m/G independent loads in batches, reading rows of Z from an LDS
// copy.  The G partial sums of a row are added in a fixed order through LDS.
#include <cstdlib>
#include <type_traits>

#include "common.h"

namespace eda {

namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int NN_NB = 8;    // output columns per workgroup (grid.y tiles the rest)
constexpr int NN_ZT = 512;  // rows of Z per LDS tile

template <typename T> __device__ __forceinline__ double ld64(const T* p) { return to_f64<T>(*p); }

// A^T B partial over one row chunk and CT consecutive 16-column tiles of A,
// nb <= 16 per z-tile: part[(chunk * m + i) * nb + j].  S: 64-row steps per
// wave.  The B rows of a step are loaded once and used for all CT tiles, so
// a wide A (many columns) does not re-read B once per 16 columns.
// blockIdx.x: row chunk, blockIdx.y: tile group + ygroups * (nb tile),
// blockIdx.z: problem.
template <typename TA, typename TB, int S, int CT, int ZT>
__device__ __forceinline__ void tn_body(const TnArgs& a, int64_t chunk, int yg, int zg) {
  const int64_t d = a.d;
  const int m = (int)a.m, nb = (int)a.nb;
  const int yt0 = yg * CT, zt0 = zg * ZT;
  if (chunk >= a.chunks || yt0 * 16 >= m || zt0 * 16 >= nb) return;
  __shared__ f64x4 red[3][CT * ZT][64];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  // B columns of the ZT tiles; a lane whose column is past nb reads column 0
  // (always valid) and contributes zeros
  const TB* bp[ZT];
  bool bok[ZT];
#pragma unroll
  for (int z = 0; z < ZT; ++z) {
    const int jz = (zt0 + z) * 16 + i;
    bok[z] = jz < nb;
    bp[z] = (const TB*)a.B + (int64_t)(bok[z] ? jz : 0) * a.ldb;
  }
  const int64_t r0 = chunk * (int64_t)(256 * S) + (int64_t)wid * (64 * S);
  const int64_t r1 = (r0 + 64 * S < d) ? r0 + 64 * S : d;
  f64x4 acc[CT * ZT];
#pragma unroll
  for (int c = 0; c < CT * ZT; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s = 0; s < S; ++s) {
    const int64_t rb = r0 + 64 * s;
    if (rb >= r1) break;
    const int64_t rs = rb + 16 * q;
    const bool full = rb + 64 <= r1;
    double bv[ZT][16];
#pragma unroll
    for (int z = 0; z < ZT; ++z)
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const bool ok = full || rs + e < r1;
        const double y = ld64(bp[z] + (ok ? rs + e : rb));
        bv[z][e] = (bok[z] && ok) ? y : 0.0;
      }
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int c0 = (yt0 + ct) * 16;
      if (c0 >= m) break;
      const bool cok = (c0 + i) < m;
      const TA* ap = (const TA*)a.A + (int64_t)(cok ? c0 + i : c0) * a.lda;
      double av[16];
      if (full) {
        if constexpr (sizeof(TA) == 1) {  // FP8: the 16 bytes of a lane in one load
          const uint4 w = *(const uint4*)((const uint8_t*)ap + rs);
          const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
          for (int e = 0; e < 16; ++e)
            av[e] = cok ? (double)fp8e4m3_decode((uint8_t)(ws[e >> 2] >> (8 * (e & 3)))) : 0.0;
        } else {
#pragma unroll
          for (int e = 0; e < 16; ++e) {
            const double x = ld64(ap + rs + e);
            av[e] = cok ? x : 0.0;
          }
        }
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const bool ok = rs + e < r1;
          const double x = ld64(ap + (ok ? rs + e : rb));
          av[e] = (cok && ok) ? x : 0.0;
        }
      }
#pragma unroll
      for (int z = 0; z < ZT; ++z) {
        if ((zt0 + z) * 16 >= nb) break;  // uniform
#pragma unroll
        for (int e = 0; e < 16; ++e)
          acc[ct * ZT + z] =
              __builtin_amdgcn_mfma_f64_16x16x4f64(av[e], bv[z][e], acc[ct * ZT + z], 0, 0, 0);
      }
    }
  }
  if (wid > 0)
#pragma unroll
    for (int c = 0; c < CT * ZT; ++c) red[wid - 1][c][lane] = acc[c];
  __syncthreads();
  if (wid == 0) {
    // accumulator layout: lane l, element v holds row 4 v + l / 16, column l % 16
    const int jj = lane & 15, ib = lane >> 4;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
#pragma unroll
      for (int z = 0; z < ZT; ++z) {
        f64x4 t = acc[ct * ZT + z];
#pragma unroll
        for (int w = 0; w < 3; ++w) t += red[w][ct * ZT + z][lane];
        const int c0 = (yt0 + ct) * 16, j0 = (zt0 + z) * 16;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int ii = 4 * v + ib;
          if (c0 + ii < m && j0 + jj < nb)
            a.part[(chunk * m + (c0 + ii)) * (int64_t)nb + (j0 + jj)] =
                (a.ascale != nullptr) ? t[v] * a.ascale[c0 + ii] : t[v];
        }
      }
    }
  }
  __syncthreads();  // red may be reused by a caller that loops over work items
}

template <typename TA, typename TB, int S, int CT, int ZT>
__global__ __launch_bounds__(256) void tn_mfma_kernel(const TnArgs* __restrict__ arr, TnArgs one,
                                                      int ygroups) {
  const TnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  tn_body<TA, TB, S, CT, ZT>(a, blockIdx.x, blockIdx.y % ygroups, blockIdx.y / ygroups);
}

// Streaming variant of tn for a narrow B (nb <= 16) and a float64/float32 A
// whose columns start on 16-byte boundaries: one 16-column tile of A per
// workgroup, the 4 waves on consecutive 64 S-row ranges.  Every load is a
// 16-byte vector load, arranged so that the 4 lanes of one column read
// consecutive 16-byte pieces (a wave instruction touches 16 column segments
// of 64 bytes), and the loads of step s + 1 are issued before the matrix-core
// products of step s, so a wave always has a step in flight.  The k slot of
// MFMA number (l, h) in lane (i, q) is row rb + 4 VW l + VW q + h (VW = 16 /
// sizeof(TA) rows per vector), the same for A and B, which is all a sum over
// rows needs.  Partial layout and chunking are those of tn_body.
template <typename T> struct Vec16 {
  static constexpr int VW = 16 / (int)sizeof(T);
  typedef T type __attribute__((ext_vector_type(VW)));
};

template <typename TA, typename TB, int S>
__device__ __forceinline__ void tn_stream_body(const TnArgs& a, int64_t chunk, int tile) {
  constexpr int VW = Vec16<TA>::VW;   // rows per A vector load (2 or 4)
  constexpr int NL = 16 / VW;         // vector loads per lane and step
  typedef typename Vec16<TA>::type VA;
  typedef TB VB __attribute__((ext_vector_type(VW)));
  const int64_t d = a.d;
  const int m = (int)a.m, nb = (int)a.nb;
  const int c0 = tile * 16;
  if (chunk >= a.chunks || c0 >= m) return;
  __shared__ f64x4 red[3][64];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const int i = lane & 15, q = lane >> 4;
  const bool cok = c0 + i < m, bok = i < nb;
  const TA* ap = (const TA*)a.A + (int64_t)(cok ? c0 + i : c0) * a.lda;
  const TB* bp = (const TB*)a.B + (int64_t)(bok ? i : 0) * a.ldb;
  const int64_t r0 = chunk * (int64_t)(256 * S) + (int64_t)wid * (64 * S);
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  double av[2][16], bv[2][16];
  // loads of step s into buffer u: element 2 l + h... (VW l + h) is row
  // rb + 4 VW l + VW q + h
  auto load = [&](int s, int u) {
    const int64_t rb = r0 + 64 * s;
    if (rb + 64 <= d) {
#pragma unroll
      for (int l = 0; l < NL; ++l) {
        const int64_t r = rb + 4 * VW * l + VW * q;
        const VA x = *(const VA*)(ap + r);
#pragma unroll
        for (int h = 0; h < VW; ++h) av[u][VW * l + h] = cok ? (double)x[h] : 0.0;
      }
      // only the lanes of B's nb columns load (the others hold zeros)
      if (bok) {
#pragma unroll
        for (int l = 0; l < NL; ++l) {
          const int64_t r = rb + 4 * VW * l + VW * q;
          const VB y = *(const VB*)(bp + r);
#pragma unroll
          for (int h = 0; h < VW; ++h) bv[u][VW * l + h] = (double)y[h];
        }
      } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) bv[u][e] = 0.0;
      }
    } else {
#pragma unroll
      for (int l = 0; l < NL; ++l)
#pragma unroll
        for (int h = 0; h < VW; ++h) {
          const int64_t r = rb + 4 * VW * l + VW * q + h;
          const bool ok = r < d;
          const double x = (double)ap[ok ? r : 0];
          const double y = (double)bp[ok ? r : 0];
          av[u][VW * l + h] = (cok && ok) ? x : 0.0;
          bv[u][VW * l + h] = (bok && ok) ? y : 0.0;
        }
    }
  };
  if (r0 < d) load(0, 0);
#pragma unroll
  for (int s = 0; s < S; ++s) {
    if (r0 + 64 * s >= d) break;
    if (s + 1 < S && r0 + 64 * (s + 1) < d) load(s + 1, (s + 1) & 1);
#pragma unroll
    for (int e = 0; e < 16; ++e)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s & 1][e], bv[s & 1][e], acc, 0, 0, 0);
  }
  if (wid > 0) red[wid - 1][lane] = acc;
  __syncthreads();
  if (wid == 0) {
    // accumulator layout: lane l, element v holds row 4 v + l / 16, column l % 16
    f64x4 t = acc;
#pragma unroll
    for (int w = 0; w < 3; ++w) t += red[w][lane];
    const int jj = lane & 15, ib = lane >> 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ii = 4 * v + ib;
      if (c0 + ii < m && jj < nb)
        a.part[(chunk * m + (c0 + ii)) * (int64_t)nb + jj] =
            (a.ascale != nullptr) ? t[v] * a.ascale[c0 + ii] : t[v];
    }
  }
}

// tn for a float64 A and B (nb <= NB, NB = 8 or 16) staged through LDS: per
// slab of 256 rows the workgroup loads its 16 columns of A and the nb columns
// of B with
// whole-wave 1 KB loads (64 lanes x 16 bytes down one column), stores them
// column-major in LDS (column stride TL_S doubles = 2 (mod 32), so the 16
// lanes of an MFMA fragment hit distinct banks), and each wave multiplies 64
// of the slab's rows on the matrix cores; the next slab is loaded into
// registers while the current one is multiplied.  Same partial layout and
// chunking (256 S rows) as tn_body.
constexpr int TL_S = 258;
template <int S, int NB>
__device__ __forceinline__ void tn_lds_body(const TnArgs& a, int64_t chunk, int tile) {
  static_assert(NB == 8 || NB == 16, "B staged as 8 or 16 columns");
  constexpr int BU = NB / 4;  // B columns loaded per wave
  typedef double d2 __attribute__((ext_vector_type(2)));
  const int64_t d = a.d;
  const int m = (int)a.m, nb = (int)a.nb;
  const int c0 = tile * 16;
  if (chunk >= a.chunks || c0 >= m) return;
  __shared__ __attribute__((aligned(32))) double As[16 * TL_S];
  __shared__ __attribute__((aligned(16))) double Bs[NB * TL_S];
  typedef const __attribute__((address_space(1))) d2* G2;
  typedef const __attribute__((address_space(1))) double* G1;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (uniform)
  const double* A = (const double*)a.A;
  const double* B = (const double*)a.B;
  const int64_t R0 = chunk * (int64_t)(256 * S);
  // this wave loads A columns c0 + wid + 4 u (u < 4) and B columns
  // BU wid + u (u < BU), rows 2 lane + 128 h of the slab (h < 2); columns
  // past m (nb) read a valid column and are zeroed by a select, so no load
  // sits behind a branch
  d2 ra[4][2], rb[BU][2];
  const double* acol[4];
  bool aok[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int c = c0 + wid + 4 * u;
    aok[u] = c < m;
    acol[u] = A + (int64_t)(aok[u] ? c : c0) * a.lda;
  }
  const double* bcol[BU];
  bool bok2[BU];
#pragma unroll
  for (int u = 0; u < BU; ++u) {
    const int j = BU * wid + u;
    bok2[u] = j < nb;
    bcol[u] = B + (int64_t)(bok2[u] ? j : 0) * a.ldb;
  }
  auto load = [&](int s) {
    const int64_t r0 = R0 + 256 * s;
    const d2 zero = {0.0, 0.0};
    if (r0 + 256 <= d) {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          ra[u][h] = *(G2)(acol[u] + r0 + 2 * lane + 128 * h);
        }
#pragma unroll
      for (int u = 0; u < BU; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          rb[u][h] = *(G2)(bcol[u] + r0 + 2 * lane + 128 * h);
        }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t r = r0 + 2 * lane + 128 * h;
          d2 v = zero;
          if (r < d) v[0] = ((G1)acol[u])[r];
          if (r + 1 < d) v[1] = ((G1)acol[u])[r + 1];
          ra[u][h] = v;
        }
#pragma unroll
      for (int u = 0; u < BU; ++u)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int64_t r = r0 + 2 * lane + 128 * h;
          d2 v = zero;
          if (r < d) v[0] = ((G1)bcol[u])[r];
          if (r + 1 < d) v[1] = ((G1)bcol[u])[r + 1];
          rb[u][h] = v;
        }
    }
  };
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  const int i = lane & 15, q = lane >> 4;
  int ns = 0;  // slabs of this chunk that hold rows < d
  while (ns < S && R0 + 256 * ns < d) ++ns;
  if (ns > 0) load(0);
  for (int s = 0; s < ns; ++s) {
    __syncthreads();  // the previous slab has been read
    // (columns past m or nb become zeros here, when their loads have landed)
    const d2 zero = {0.0, 0.0};
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        *(d2*)(As + (wid + 4 * u) * TL_S + 2 * lane + 128 * h) = aok[u] ? ra[u][h] : zero;
#pragma unroll
    for (int u = 0; u < BU; ++u)
#pragma unroll
      for (int h = 0; h < 2; ++h)
        *(d2*)(Bs + (BU * wid + u) * TL_S + 2 * lane + 128 * h) = bok2[u] ? rb[u][h] : zero;
    __syncthreads();
    if (s + 1 < ns) load(s + 1);
    const double* ac = As + i * TL_S + 64 * wid + q;
    const double* bc = Bs + (i < NB ? i : 0) * TL_S + 64 * wid + q;
#pragma unroll
    for (int e = 0; e < 16; ++e) {
      const double x = ac[4 * e];
      const double y = (i < nb) ? bc[4 * e] : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
    }
  }
  // the 4 waves' sums (each over its quarter of every slab) meet in LDS
  __syncthreads();
  f64x4* red = (f64x4*)As;
  if (wid > 0) red[(wid - 1) * 64 + lane] = acc;
  __syncthreads();
  if (wid == 0) {
    f64x4 t = acc;
#pragma unroll
    for (int w = 0; w < 3; ++w) t += red[w * 64 + lane];
    const int jj = lane & 15, ib = lane >> 4;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int ii = 4 * v + ib;
      if (c0 + ii < m && jj < nb)
        a.part[(chunk * m + (c0 + ii)) * (int64_t)nb + jj] =
            (a.ascale != nullptr) ? t[v] * a.ascale[c0 + ii] : t[v];
    }
  }
}

// tn for a narrow A (FP8 E4M3 or bfloat16 codes) and a float32 or bfloat16
// B (nb <= 8) on the bfloat16 matrix cores.  A workgroup owns 64 columns of
// A (4 tiles of 16) and one row chunk of 256 S rows; slabs of 32 KB of A
// (and the matching rows of B) are staged through LDS with whole-wave
// 16-byte loads (32 lanes down each column), and each wave multiplies a
// quarter of every slab's rows for all 4 tiles.  FP8 codes are widened by
// the hardware E4M3 -> float32 conversion (exact) and truncated to bfloat16
// (exact: E4M3 values have 4 significant bits); a float32 B is split into
// three bfloat16 terms hi + mid + lo (exact to float32's precision), a
// bfloat16 B is used as it is, so every product of
// v_mfma_f32_16x16x32_bf16 is exact and each 32-row step is accumulated in
// float32 from zero and then added into float64 accumulators.  The 4 waves' sums meet in LDS in a fixed
// order, scaled by the per-column scales on output (tn_body's layout).
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ __bf16 bf16_of_bits(uint16_t u) {
  __bf16 r;
  __builtin_memcpy(&r, &u, 2);
  return r;
}
// float32 -> bfloat16 with round to nearest even (finite inputs)
__device__ __forceinline__ uint16_t bf16_rne_f32(float x) {
  const uint32_t u = __float_as_uint(x);
  return (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
// 8 E4M3 codes (two words) -> 8 bfloat16 values, exact
__device__ __forceinline__ bf16x8 fp8x8_to_bf16(uint32_t w0, uint32_t w1) {
  bf16x8 r;
  const uint32_t ws[2] = {w0, w1};
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)ws[q], false);
    const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)ws[q], true);
    r[4 * q + 0] = bf16_of_bits((uint16_t)(__float_as_uint(lo.x) >> 16));
    r[4 * q + 1] = bf16_of_bits((uint16_t)(__float_as_uint(lo.y) >> 16));
    r[4 * q + 2] = bf16_of_bits((uint16_t)(__float_as_uint(hi.x) >> 16));
    r[4 * q + 3] = bf16_of_bits((uint16_t)(__float_as_uint(hi.y) >> 16));
  }
  return r;
}

template <typename TA, typename TB, int S>
__device__ __forceinline__ void tn_narrow_body(const TnArgs& a, int64_t chunk, int grp) {
  constexpr int SZ = (int)sizeof(TA);
  constexpr int BZ = (int)sizeof(TB);        // 4 (float32 block) or 2 (bfloat16 block)
  constexpr int SR = 32768 / (64 * SZ);      // rows per slab: 512 (FP8), 256 (bfloat16)
  constexpr int CB = SR * SZ;                // bytes per column per slab (512)
  constexpr int CS = CB + 16;                // LDS column stride (bytes)
  constexpr int BCB = SR * BZ;               // bytes per column of B per slab
  constexpr int BS = BCB + 16;               // LDS column stride of B (bytes)
  constexpr int NSL = 256 * S / SR;          // slabs per chunk
  constexpr int WR = SR / 4;                 // rows per wave per slab
  constexpr int NKS = WR / 32;               // 32-row MFMA steps per wave per slab
  constexpr int BPC = BCB / 16;              // 16-byte pieces of B per column per slab
  constexpr int NBL = 8 * BPC / 256;         // 16-byte loads of B per thread per slab
  static_assert(NSL >= 1 && (256 * S) % SR == 0, "a chunk must hold whole slabs");
  static_assert(NBL >= 1 && (8 * BPC) % 256 == 0, "B slab split over the workgroup");
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  typedef const __attribute__((address_space(1))) u32x4* G4;

  const int64_t d = a.d;
  const int m = (int)a.m, nb = (int)a.nb;
  const int c0 = grp * 64;
  if (chunk >= a.chunks || c0 >= m) return;
  __shared__ __attribute__((aligned(16))) uint8_t As[64 * CS];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[8 * BS];
  static_assert(3 * 4 * 4 * 64 * 8 <= 64 * CS, "the wave sums must fit in the slab buffer");
  double(*red)[4][4][64] = (double(*)[4][4][64])As;  // reused after the last slab
  const int tid = threadIdx.x, lane = tid & 63;
  const int wid = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int i = lane & 15, kq = lane >> 4;
  const uint8_t* A = (const uint8_t*)a.A;
  const uint8_t* B = (const uint8_t*)a.B;
  const int64_t ldb_b = a.ldb * BZ;
  const int64_t lda_b = a.lda * SZ;
  const int64_t R0 = chunk * (int64_t)(256 * S);
  // loads of a slab: A element e = tid + 256 u (u < 8) is column e / 32,
  // bytes 16 (e % 32) .. + 15 of that column's CB; B piece g = tid + 256 u
  // (u < NBL) is column g / BPC, bytes 16 (g % BPC) .. + 15 of its BCB
  u32x4 ra[8];
  u32x4 rbv[NBL];
  const u32x4 z4 = {0u, 0u, 0u, 0u};
  auto load = [&](int sl) {
    const int64_t r0 = R0 + (int64_t)sl * SR;
    const bool full = r0 + SR <= d;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      const int cl = e >> 5, off = (e & 31) * 16;
      const int c = c0 + cl;
      const uint8_t* p = A + (int64_t)(c < m ? c : c0) * lda_b + r0 * SZ + off;
      if (full) {
        ra[u] = *(G4)p;
      } else {
        // pieces wholly past d read as zero; the piece holding row d - 1 is
        // read byte by byte up to it
        const int64_t rfirst = r0 + off / SZ;
        u32x4 v = z4;
        if (rfirst + 16 / SZ <= d) {
          v = *(G4)p;
        } else if (rfirst < d) {
          const int keep = (int)((d - rfirst) * SZ);  // bytes of rows < d in this piece
          uint8_t bytes[16];
          for (int q = 0; q < 16; ++q)
            bytes[q] = (q < keep) ? ((const __attribute__((address_space(1))) uint8_t*)p)[q] : 0;
          __builtin_memcpy(&v, bytes, 16);
        }
        ra[u] = v;
      }
    }
#pragma unroll
    for (int u = 0; u < NBL; ++u) {
      const int g = tid + 256 * u;
      const int col = g / BPC, off = (g % BPC) * 16;
      const int cc = col < nb ? col : 0;
      const uint8_t* p = B + (int64_t)cc * ldb_b + r0 * BZ + off;
      u32x4 v = z4;
      const int64_t rfirst = r0 + off / BZ;
      if (full || rfirst + 16 / BZ <= d) {
        v = *(G4)p;
      } else if (rfirst < d) {
        const int keep = (int)((d - rfirst) * BZ);  // bytes of rows < d in this piece
        uint8_t bytes[16];
        for (int q = 0; q < 16; ++q)
          bytes[q] = (q < keep) ? ((const __attribute__((address_space(1))) uint8_t*)p)[q] : 0;
        __builtin_memcpy(&v, bytes, 16);
      }
      rbv[u] = (col < nb) ? v : z4;
    }
  };
  double acc[4][4];
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[t][v] = 0.0;
  int nsl = 0;
  while (nsl < NSL && R0 + (int64_t)nsl * SR < d) ++nsl;
  if (nsl > 0) load(0);
  for (int sl = 0; sl < nsl; ++sl) {
    __syncthreads();  // the previous slab has been read
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = tid + 256 * u;
      const int cl = e >> 5, off = (e & 31) * 16;
      *(u32x4*)(As + cl * CS + off) = (c0 + cl < m) ? ra[u] : z4;
    }
#pragma unroll
    for (int u = 0; u < NBL; ++u) {
      const int g = tid + 256 * u;
      const int col = g / BPC, off = (g % BPC) * 16;
      *(u32x4*)(Bs + col * BS + off) = rbv[u];
    }
    __syncthreads();
    if (sl + 1 < nsl) load(sl + 1);
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int rl = wid * WR + 32 * ks + 8 * kq;  // first of this lane's 8 rows in the slab
      // B: rows rl .. + 7 of column i (zero past nb and past d); a float32
      // block is split into three bfloat16 terms, a bfloat16 one is used as is
      constexpr int NT = (BZ == 4) ? 3 : 1;
      bf16x8 bt[NT];
      {
        const uint8_t* bp = Bs + (i < 8 ? i : 0) * BS + rl * BZ;
        if constexpr (BZ == 4) {
          const f32x4 x0 = *(const f32x4*)bp;
          const f32x4 x1 = *(const f32x4*)(bp + 16);
          float bv[8];
#pragma unroll
          for (int e = 0; e < 4; ++e) {
            bv[e] = i < 8 ? x0[e] : 0.0f;
            bv[4 + e] = i < 8 ? x1[e] : 0.0f;
          }
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const uint16_t hb = bf16_rne_f32(bv[e]);
            const float r1 = bv[e] - __uint_as_float((uint32_t)hb << 16);
            const uint16_t mb = bf16_rne_f32(r1);
            const float r2 = r1 - __uint_as_float((uint32_t)mb << 16);
            bt[0][e] = bf16_of_bits(hb);
            bt[NT - 2][e] = bf16_of_bits(mb);
            bt[NT - 1][e] = bf16_of_bits(bf16_rne_f32(r2));
          }
        } else {
          const u32x4 w = i < 8 ? *(const u32x4*)bp : z4;
          __builtin_memcpy(&bt[0], &w, 16);
        }
      }
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const uint8_t* ap = As + (16 * t + i) * CS + rl * SZ;
        bf16x8 av;
        if constexpr (SZ == 1) {
          const uint2 w = *(const uint2*)ap;
          av = fp8x8_to_bf16(w.x, w.y);
        } else {
          const u32x4 w = *(const u32x4*)ap;
          __builtin_memcpy(&av, &w, 16);
        }
        f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < NT; ++q)
          c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bt[q], c, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; ++v) acc[t][v] += (double)c[v];
      }
    }
  }
  // fixed-order sum of the 4 waves (each over its quarter of every slab)
  __syncthreads();  // the last slab has been read
  if (wid > 0)
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) red[wid - 1][t][v][lane] = acc[t][v];
  __syncthreads();
  if (wid == 0) {
    // accumulator element v of lane l: row 4 (l / 16) + v of the tile, column l % 16
    const int jj = lane & 15, ib = lane >> 4;
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double sum = ((acc[t][v] + red[0][t][v][lane]) + red[1][t][v][lane]) +
                           red[2][t][v][lane];
        const int col = c0 + 16 * t + 4 * ib + v;
        if (col < m && jj < nb)
          a.part[(chunk * m + col) * (int64_t)nb + jj] =
              (a.ascale != nullptr) ? sum * a.ascale[col] : sum;
      }
  }
}

template <typename TA, typename TB, int S>
__global__ __launch_bounds__(256) void tn_narrow_kernel(const TnArgs* __restrict__ arr,
                                                        TnArgs one) {
  const TnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  tn_narrow_body<TA, TB, S>(a, blockIdx.x, blockIdx.y);
}

template <int S, int NB>
__global__ __launch_bounds__(256) void tn_lds_kernel(const TnArgs* __restrict__ arr, TnArgs one) {
  const TnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  tn_lds_body<S, NB>(a, blockIdx.x, blockIdx.y);
}

template <typename TA, typename TB, int S>
__global__ __launch_bounds__(256) void tn_stream_kernel(const TnArgs* __restrict__ arr,
                                                        TnArgs one) {
  const TnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  tn_stream_body<TA, TB, S>(a, blockIdx.x, blockIdx.y);
}

// Sum of the chunk partials, fixed order: wave w adds chunks w, w+4, ... of
// 64 outputs, then the 4 wave sums are added in order.
__device__ __forceinline__ void reduce_body(const ReduceArgs& a, int64_t bx) {
  const int64_t mn = a.m * a.nb;
  if (bx * 64 >= mn) return;
  __shared__ double red[3][64];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t chunks = a.chunks;
  const double* __restrict__ part = a.part;
  const int64_t e = bx * 64 + lane;
  const int64_t ee = e < mn ? e : mn - 1;
  const int64_t i = e / a.nb, j = e - i * a.nb;
  // the accumulated output is read before the partials, so that its memory
  // round trip overlaps theirs
  const bool toc2 = a.mc >= 0 && i >= a.mc;
  const double cprev = (wid == 0 && e < mn && a.C != nullptr && !toc2 && a.beta != 0.0)
                           ? a.C[i + j * a.ldc]
                           : 0.0;
  // 16 loads in flight per lane; chunks w, w+4, ... added in order
  double s = 0.0;
  for (int64_t c0 = wid; c0 < chunks; c0 += 64) {
    double v[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) {
      const int64_t c = c0 + 4 * u;
      v[u] = (c < chunks) ? part[c * mn + ee] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 16; ++u)
      if (c0 + 4 * u < chunks) s += v[u];
  }
  if (wid > 0) red[wid - 1][lane] = s;
  __syncthreads();
  if (wid == 0 && e < mn) {
    s += red[0][lane];
    s += red[1][lane];
    s += red[2][lane];
    if (toc2)
      a.C2[(i - a.mc) + j * a.ldc2] = s;
    else if (a.C != nullptr)
      a.C[i + j * a.ldc] = a.beta * cprev + a.alpha * s;
    if (a.Z != nullptr) a.Z[i * a.ldz + j] = a.zalpha * s;
  }
  __syncthreads();  // red may be reused by a caller that loops over work items
}

__global__ __launch_bounds__(256) void reduce_partials_kernel(const ReduceArgs* __restrict__ arr,
                                                              ReduceArgs one) {
  const ReduceArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  reduce_body(a, blockIdx.x);
}

template <typename TA, typename TV, typename TO, typename ACC, int R, int BATCH>
__device__ __forceinline__ void nn_body(const NnArgs& a, int64_t bx, int by) {
  const int64_t d = a.d;
  const int m = (int)a.m, nb = (int)a.nb;
  const int j0 = by * NN_NB;
  if (bx * R >= d || j0 >= nb) return;
  constexpr int G = 256 / R;
  __shared__ ACC zs[NN_ZT * NN_NB];
  __shared__ ACC red[256 * (NN_NB + 1)];
  const int tid = threadIdx.x;
  const int rl = tid % R, g = tid / R;
  const int64_t r = bx * R + rl;
  const int64_t lda = a.lda;
  const TA* ar = (const TA*)a.A + (r < d ? r : d - 1);  // rows past d read row d-1, never stored
  const TV* V = (const TV*)a.V;
  TO* Out = (TO*)a.Out;
  // the operands of the output step are loaded now, so that their memory
  // round trip overlaps the main loop (each thread reads only the V entries
  // it overwrites in Out, so V == Out is safe)
  constexpr int NO = (R * NN_NB + 255) / 256;
  const double alpha = (a.alpha_p != nullptr) ? *a.alpha_p : a.alpha;
  double vpre[NO];
  int mpre[NO];
#pragma unroll
  for (int q = 0; q < NO; ++q) {
    const int e = tid + 256 * q;
    const int rr = e % R, j = e / R;
    const int64_t row = bx * R + rr;
    const bool ok = e < R * NN_NB && row < d && j0 + j < nb;
    vpre[q] = (ok && V != nullptr) ? to_f64<TV>(V[row + (int64_t)(j0 + j) * a.ldv]) : 0.0;
    mpre[q] = (ok && a.mask != nullptr) ? a.mask[j0 + j] : 0;
  }
  ACC acc[NN_NB];
#pragma unroll
  for (int j = 0; j < NN_NB; ++j) acc[j] = ACC(0);
  for (int t0 = 0; t0 < m; t0 += NN_ZT) {
    const int tn = (m - t0 < NN_ZT) ? m - t0 : NN_ZT;
    __syncthreads();
    for (int e = tid; e < tn * NN_NB; e += 256) {
      const int i = e / NN_NB, j = e - i * NN_NB;
      double z = (j0 + j < nb) ? a.Z[(int64_t)(t0 + i) * a.ldz + j0 + j] : 0.0;
      if (a.ascale != nullptr) z *= a.ascale[t0 + i];
      zs[e] = (ACC)z;
    }
    __syncthreads();
    // BATCH loads issued together per step, the tail guarded (one memory
    // round trip per BATCH columns of A)
    for (int i = g; i < tn; i += BATCH * G) {
      ACC av[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int ii = i + u * G;
        av[u] = (ii < tn) ? to_acc<ACC>(ar[(int64_t)(t0 + ii) * lda]) : ACC(0);
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int ii = i + u * G;
        if (ii < tn) {
          const ACC* zr = zs + ii * NN_NB;
#pragma unroll
          for (int j = 0; j < NN_NB; ++j) acc[j] += av[u] * zr[j];
        }
      }
    }
  }
#pragma unroll
  for (int j = 0; j < NN_NB; ++j) red[tid * (NN_NB + 1) + j] = acc[j];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NO; ++q) {
    const int e = tid + 256 * q;
    if (e >= R * NN_NB) continue;
    const int rr = e % R, j = e / R;
    const int64_t row = bx * R + rr;
    if (row >= d || j0 + j >= nb) continue;
    ACC sacc = ACC(0);
    for (int u = 0; u < G; ++u) sacc += red[(u * R + rr) * (NN_NB + 1) + j];
    double o = (double)sacc;
    if (alpha != 0.0) o += alpha * vpre[q];
    if (mpre[q] != 0) o = masked_gauss(a.seed, (int64_t)(j0 + j) * d + row);
    const int64_t oi = a.out_row ? row * a.ldo + (j0 + j) : row + (int64_t)(j0 + j) * a.ldo;
    Out[oi] = from_f64<TO>(o);
  }
  __syncthreads();  // red and zs may be reused by a caller that loops over work items
}

template <typename TA, typename TV, typename TO, typename ACC, int R, int BATCH>
__global__ __launch_bounds__(256) void nn_kernel(const NnArgs* __restrict__ arr, NnArgs one) {
  const NnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  nn_body<TA, TV, TO, ACC, R, BATCH>(a, blockIdx.x, blockIdx.y);
}

// Streaming variant of nn for a long A (float64 or float32) with 16-byte
// aligned columns and at most NB output columns (NB = 8 or 16), all in one
// workgroup column: a workgroup owns 64 VW rows (VW = 16 / sizeof(TA): each
// lane reads VW consecutive rows of a column with one 16-byte load, so a
// wave instruction moves 1 KB of one column), each of its 4 waves takes
// every fourth column, NS_B column loads in flight per wave.  The row of Z that
// multiplies a column is the same for the whole wave, so it is read with
// scalar loads (through the scalar cache) straight from global memory: no
// LDS staging and no barrier while A streams.  The 4 waves' sums meet in LDS
// in a fixed order.  Every workgroup reads all of A's columns for its rows
// before it writes those rows, so Out may be A itself (columns 0 .. nb, same
// leading dimension).  With kcols > 0 the columns are split into groups of
// kcols (blockIdx.y = group) and every group writes its partial product,
// row-major, to Out + group * d * nb (ldo = nb, no V term): a fixed-order
// reduction over the groups finishes it.
constexpr int NS_B = 8;
constexpr int NS_RED = 4096;  // doubles of LDS for the reduction over the 4 waves
typedef const __attribute__((address_space(4))) double* ConstF64;

// A 64-bit value made provably wave-uniform (the argument structs are read
// through generic pointers, whose loads the compiler must treat as
// per-lane): lets loads through it become scalar loads.
__device__ __forceinline__ uint64_t wave_uniform64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Columns [k0, k1) of A times the matching rows of Z, accumulated into acc:
// wave w takes the columns k1 - 1 - w - 4 u, from the last column down (the
// P^T V pass that precedes a product walks P's columns upwards, so its last
// columns may still be in the Infinity Cache), NS_B loads per batch issued
// before the batch's products.  FULL: every row of the workgroup is < d (plain
// vector loads); else rows >= d read as zero.  NBFULL: nb == NB, whole Z
// rows by wide scalar loads; else Z entries are read at indices below nb
// only (one guarded load each), so a Z of exactly m rows of nb entries is
// never overrun.
template <typename TA, int NB, bool FULL, bool NBFULL>
__device__ __forceinline__ void nn_stream_cols(const TA* __restrict__ ar, int64_t lda, int64_t row0,
                                               int64_t d, int k0, int k1, int w,
                                               const double* __restrict__ Z, int64_t ldz, int nb,
                                               double (&acc)[Vec16<TA>::VW][NB]) {
  constexpr int VW = Vec16<TA>::VW;
  typedef typename Vec16<TA>::type VA;
  typedef const __attribute__((address_space(1))) VA* GVA;
  typedef const __attribute__((address_space(1))) TA* GTA;
  const int nloc = (k1 - k0 - w + 3) / 4;  // columns of this wave (uniform)
  for (int c = 0; c < nloc; c += NS_B) {
    // loads of the batch first (columns past the wave's last are clamped to
    // its first and weighted by zero), then the products
    VA raw[NS_B];
#pragma unroll
    for (int u = 0; u < NS_B; ++u) {
      const int cc = (c + u < nloc) ? c + u : 0;
      const TA* colp = ar + (int64_t)(k1 - 1 - w - 4 * cc) * lda;
      if constexpr (FULL) {
        raw[u] = *(GVA)colp;
      } else {
#pragma unroll
        for (int h = 0; h < VW; ++h) raw[u][h] = (row0 + h < d) ? ((GTA)colp)[h] : (TA)0;
      }
    }
#pragma unroll
    for (int u = 0; u < NS_B; ++u) {
      const bool live = c + u < nloc;
      const int64_t col = k1 - 1 - w - 4 * (live ? c + u : 0);
      const ConstF64 zp = (ConstF64)(Z + col * ldz);
      double zr[NB];
      if constexpr (NBFULL) {
#pragma unroll
        for (int j = 0; j < NB; ++j) zr[j] = zp[j];
      } else {
#pragma unroll
        for (int j = 0; j < NB; ++j) zr[j] = (j < nb) ? zp[j < nb ? j : 0] : 0.0;
      }
      const double f = live ? 1.0 : 0.0;
#pragma unroll
      for (int h = 0; h < VW; ++h) {
        const double x = (double)raw[u][h] * f;
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[h][j] += x * zr[j];
      }
    }
  }
}

template <typename TA, typename TV, typename TO, int NB>
__device__ __forceinline__ void nn_stream_body(const NnArgs& a, int64_t bx, int by) {
  constexpr int VW = Vec16<TA>::VW;
  constexpr int R = 64 * VW;  // rows per workgroup
  const int64_t d = a.d;
  const int m = __builtin_amdgcn_readfirstlane((int)a.m);
  const int nb = __builtin_amdgcn_readfirstlane((int)a.nb);
  const int kcols = __builtin_amdgcn_readfirstlane((int)a.kcols);
  const bool split = kcols > 0;
  const int k0 = split ? by * kcols : 0;
  const int k1 = split ? min(m, k0 + kcols) : m;
  if (bx * R >= d || k0 >= k1) return;
  __shared__ double zs[NS_RED];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave index (uniform)
  const int64_t row0 = bx * R + (int64_t)lane * VW;  // first of this lane's VW rows
  const bool full = bx * R + R <= d;                  // every row of the workgroup < d
  const TA* ar = (const TA*)a.A + (row0 < d ? row0 : 0);
  double acc[VW][NB];
#pragma unroll
  for (int h = 0; h < VW; ++h)
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[h][j] = 0.0;
  const double* Z = (const double*)wave_uniform64((uint64_t)a.Z);
  const int64_t ldz = (int64_t)wave_uniform64((uint64_t)a.ldz);
  if (nb == NB) {
    if (full)
      nn_stream_cols<TA, NB, true, true>(ar, a.lda, row0, d, k0, k1, w, Z, ldz, nb, acc);
    else
      nn_stream_cols<TA, NB, false, true>(ar, a.lda, row0, d, k0, k1, w, Z, ldz, nb, acc);
  } else {
    if (full)
      nn_stream_cols<TA, NB, true, false>(ar, a.lda, row0, d, k0, k1, w, Z, ldz, nb, acc);
    else
      nn_stream_cols<TA, NB, false, false>(ar, a.lda, row0, d, k0, k1, w, Z, ldz, nb, acc);
  }
  // the 4 waves' sums meet in LDS, JP columns at a time
  constexpr int JP = (NS_RED / (4 * R) < NB) ? NS_RED / (4 * R) : NB;
  static_assert(JP >= 1 && NB % JP == 0 && (R * JP) % 256 == 0, "reduction passes");
  const double alpha = split ? 0.0 : ((a.alpha_p != nullptr) ? *a.alpha_p : a.alpha);
  const TV* V = (const TV*)a.V;
  TO* Out = (TO*)a.Out;
  if (split) Out += (int64_t)by * d * nb;
#pragma unroll
  for (int jp = 0; jp < NB; jp += JP) {
    __syncthreads();
#pragma unroll
    for (int h = 0; h < VW; ++h)
#pragma unroll
      for (int j = 0; j < JP; ++j) zs[(w * R + lane * VW + h) * JP + j] = acc[h][jp + j];
    __syncthreads();
    // output element e = tid + 256 q: row e % R of the workgroup, column jp + e / R
    constexpr int NO = R * JP / 256;
#pragma unroll
    for (int qq = 0; qq < NO; ++qq) {
      const int e = tid + 256 * qq;
      const int rr = e % R, jl = e / R, j = jp + jl;
      const int64_t row = bx * R + rr;
      if (row >= d || j >= nb) continue;
      double o = ((zs[(0 * R + rr) * JP + jl] + zs[(1 * R + rr) * JP + jl]) +
                  zs[(2 * R + rr) * JP + jl]) + zs[(3 * R + rr) * JP + jl];
      if (alpha != 0.0 && V != nullptr) o += alpha * to_f64<TV>(V[row + (int64_t)j * a.ldv]);
      if (!split && a.mask != nullptr && a.mask[j] != 0)
        o = masked_gauss(a.seed, (int64_t)j * d + row);
      const int64_t oi = (split || a.out_row) ? row * (split ? nb : a.ldo) + j
                                              : row + (int64_t)j * a.ldo;
      Out[oi] = from_f64<TO>(o);
    }
  }
}

template <typename TA, typename TV, typename TO, int NB>
__global__ __launch_bounds__(256) void nn_stream_kernel(const NnArgs* __restrict__ arr, NnArgs one) {
  const NnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  nn_stream_body<TA, TV, TO, NB>(a, blockIdx.x, blockIdx.y);
}

// nn for wide outputs (nb > 8): NNW_NB output columns per workgroup, so that
// A streams once per 40 columns instead of once per 8 (the Ritz blocks of
// the final stage, restarts and orthonormalisation of t columns).  Z tiles
// of NNW_ZT rows in LDS; the partial sums of the G = 256 / R column groups
// meet in LDS eight output columns at a time, in a fixed order.
constexpr int NNW_NB = 40;
constexpr int NNW_ZT = 96;
template <typename TA, typename TV, typename TO, typename ACC, int R, int BATCH>
__device__ __forceinline__ void nn_wide_body(const NnArgs& a, int64_t bx, int by) {
  static_assert(R == 32 || R == 64, "an 8-column chunk must fill whole output slots");
  constexpr int NB = NNW_NB, G = 256 / R, QC = 8 * R / 256, NO = R * NB / 256;
  const int64_t d = a.d;
  const int m = (int)a.m, nb = (int)a.nb;
  const int j0 = by * NB;
  if (bx * R >= d || j0 >= nb) return;
  __shared__ ACC zs[NNW_ZT * NB];
  __shared__ ACC red[256 * 9];
  const int tid = threadIdx.x;
  const int rl = tid % R, g = tid / R;
  const int64_t r = bx * R + rl;
  const int64_t lda = a.lda;
  const TA* ar = (const TA*)a.A + (r < d ? r : d - 1);  // rows past d read row d-1, never stored
  const TV* V = (const TV*)a.V;
  TO* Out = (TO*)a.Out;
  // output slot q of a thread: e = tid + 256 q, row e % R, column e / R;
  // each thread reads only the V entries it overwrites, so V == Out is safe
  const double alpha = (a.alpha_p != nullptr) ? *a.alpha_p : a.alpha;
  double vpre[NO];
  int mpre[NO];
#pragma unroll
  for (int q = 0; q < NO; ++q) {
    const int e = tid + 256 * q;
    const int rr = e % R, j = e / R;
    const int64_t row = bx * R + rr;
    const bool ok = row < d && j0 + j < nb;
    vpre[q] = (ok && V != nullptr) ? to_f64<TV>(V[row + (int64_t)(j0 + j) * a.ldv]) : 0.0;
    mpre[q] = (ok && a.mask != nullptr) ? a.mask[j0 + j] : 0;
  }
  ACC acc[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) acc[j] = ACC(0);
  for (int t0 = 0; t0 < m; t0 += NNW_ZT) {
    const int tn = (m - t0 < NNW_ZT) ? m - t0 : NNW_ZT;
    __syncthreads();
    for (int e = tid; e < tn * NB; e += 256) {
      const int i = e / NB, j = e - i * NB;
      double z = (j0 + j < nb) ? a.Z[(int64_t)(t0 + i) * a.ldz + j0 + j] : 0.0;
      if (a.ascale != nullptr) z *= a.ascale[t0 + i];
      zs[e] = (ACC)z;
    }
    __syncthreads();
    for (int i = g; i < tn; i += BATCH * G) {
      ACC av[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int ii = i + u * G;
        av[u] = (ii < tn) ? to_acc<ACC>(ar[(int64_t)(t0 + ii) * lda]) : ACC(0);
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int ii = i + u * G;
        if (ii < tn) {
          const ACC* zr = zs + ii * NB;
#pragma unroll
          for (int j = 0; j < NB; ++j) acc[j] += av[u] * zr[j];
        }
      }
    }
  }
#pragma unroll
  for (int c8 = 0; c8 < NB / 8; ++c8) {
    __syncthreads();  // the previous chunk has been read
#pragma unroll
    for (int j = 0; j < 8; ++j) red[tid * 9 + j] = acc[8 * c8 + j];
    __syncthreads();
#pragma unroll
    for (int qq = 0; qq < QC; ++qq) {
      const int q = c8 * QC + qq;
      const int e = tid + 256 * q;
      const int rr = e % R, j = e / R;  // 8 c8 <= j < 8 c8 + 8
      const int64_t row = bx * R + rr;
      if (row >= d || j0 + j >= nb) continue;
      ACC sacc = ACC(0);
      for (int u = 0; u < G; ++u) sacc += red[(u * R + rr) * 9 + (j - 8 * c8)];
      double o = (double)sacc;
      if (alpha != 0.0) o += alpha * vpre[q];
      if (mpre[q] != 0) o = masked_gauss(a.seed, (int64_t)(j0 + j) * d + row);
      const int64_t oi = a.out_row ? row * a.ldo + (j0 + j) : row + (int64_t)(j0 + j) * a.ldo;
      Out[oi] = from_f64<TO>(o);
    }
  }
  __syncthreads();
}

template <typename TA, typename TV, typename TO, typename ACC, int R, int BATCH>
__global__ __launch_bounds__(256) void nn_wide_kernel(const NnArgs* __restrict__ arr, NnArgs one) {
  const NnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  nn_wide_body<TA, TV, TO, ACC, R, BATCH>(a, blockIdx.x, blockIdx.y);
}

// nn for wide outputs over a long float64 A on the matrix cores: a wave owns
// 16 rows of A and CTN 16-column tiles of the output, a workgroup 64 rows;
// Z is staged in LDS in tiles of NNM_KT rows shared by the four waves, and
// each A entry, loaded once, feeds CTN v_mfma_f64_16x16x4f64.  Operand
// layout: A(i, k) at lane i + 16 k, Z(k, j) at lane j + 16 k; accumulator
// element v of lane l is Out(4 v + l / 16, l % 16).  For Out = alpha V + A Z
// without mask, column scales or row-major output.
constexpr int NNM_KT = 32;
template <int CTN>
__global__ __launch_bounds__(256) void nn_mfma_kernel(const NnArgs* __restrict__ arr, NnArgs one) {
  const NnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  const int64_t d = a.d;
  const int m = (int)a.m, nb = (int)a.nb;
  const int64_t row0 = (int64_t)blockIdx.x * 64;
  const int j0 = blockIdx.y * 16 * CTN;
  if (row0 >= d || j0 >= nb) return;
  constexpr int ZW = 16 * CTN;  // Z columns staged per tile
  __shared__ double zs[NNM_KT * ZW];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int li = lane & 15, lk = lane >> 4;
  const int64_t r = row0 + wid * 16 + li;
  const double* ar = (const double*)a.A + (r < d ? r : d - 1);  // rows past d: never stored
  const int64_t lda = a.lda;
  f64x4 acc[CTN];
#pragma unroll
  for (int c = 0; c < CTN; ++c) acc[c] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < m; k0 += NNM_KT) {
    // this tile's A entries first, so that their round trip overlaps the
    // staging of Z
    double av[NNM_KT / 4];
#pragma unroll
    for (int q = 0; q < NNM_KT / 4; ++q) {
      const int k = k0 + 4 * q + lk;
      av[q] = (k < m) ? ar[(int64_t)k * lda] : 0.0;
    }
    __syncthreads();  // the previous tile has been read
    for (int e = tid; e < NNM_KT * ZW; e += 256) {
      const int kk = e / ZW, j = e - kk * ZW;
      const int k = k0 + kk;
      zs[e] = (k < m && j0 + j < nb) ? a.Z[(int64_t)k * a.ldz + j0 + j] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NNM_KT / 4; ++q) {
      const double* zr = zs + (4 * q + lk) * ZW + li;
#pragma unroll
      for (int c = 0; c < CTN; ++c)
        if (j0 + 16 * c < nb)  // uniform
          acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[q], zr[16 * c], acc[c], 0, 0, 0);
    }
  }
  const double alpha = (a.alpha_p != nullptr) ? *a.alpha_p : a.alpha;
  const double* V = (const double*)a.V;
  double* Out = (double*)a.Out;
#pragma unroll
  for (int c = 0; c < CTN; ++c) {
    const int j = j0 + 16 * c + li;
    if (j >= nb) continue;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int64_t row = row0 + wid * 16 + 4 * v + lk;
      if (row >= d) continue;
      double o = acc[c][v];
      if (alpha != 0.0 && V != nullptr) o += alpha * V[row + (int64_t)j * a.ldv];
      Out[row + (int64_t)j * a.ldo] = o;
    }
  }
}

// nn for a narrow A (FP8 or bfloat16 entries).  A lane owns 8 consecutive
// rows and reads them with one 8-byte (FP8) or 16-byte (bfloat16) load per
// column: a wave instruction then moves 512 or 1024 contiguous bytes
// instead of one entry per lane.  Lane (rl = l % 16, gq = l / 16) of wave w
// takes rows 8 rl .. 8 rl + 7 of the workgroup's 128 and the columns
// j = g mod 16, g = 4 w + gq; the 4 column groups of a wave are summed by
// lane exchanges, the 4 waves through LDS, both in a fixed order.
constexpr int NNN_R = 128;  // rows per workgroup of the narrow nn
template <typename TA, typename TV, typename TO, typename ACC>
__device__ __forceinline__ void nn_narrow_body(const NnArgs& a, int64_t bx, int by) {
  constexpr int NR = 8, BATCH = 8, G = 16;
  using RAW = typename std::conditional<sizeof(TA) == 1, uint2, uint4>::type;
  const int64_t d = a.d;
  const int m = (int)a.m, nb = (int)a.nb;
  const int j0 = by * NN_NB;
  if (bx * NNN_R >= d || j0 >= nb) return;
  __shared__ ACC zs[NN_ZT * NN_NB];
  __shared__ ACC red[4][NNN_R][NN_NB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int rl = lane & 15, gq = lane >> 4, g = 4 * w + gq;
  const int64_t row0 = bx * NNN_R + 8 * rl;
  const bool rok = row0 < a.lda;  // rows d .. lda-1 of A are zero padding
  const int64_t lda = a.lda;
  const char* abase = (const char*)a.A + row0 * (int64_t)sizeof(TA);
  const TV* V = (const TV*)a.V;
  TO* Out = (TO*)a.Out;
  constexpr int NO = (NNN_R * NN_NB + 255) / 256;
  const double alpha = (a.alpha_p != nullptr) ? *a.alpha_p : a.alpha;
  double vpre[NO];
  int mpre[NO];
#pragma unroll
  for (int q = 0; q < NO; ++q) {
    const int e = tid + 256 * q;
    const int rr = e % NNN_R, j = e / NNN_R;
    const int64_t row = bx * NNN_R + rr;
    const bool ok = row < d && j0 + j < nb;
    vpre[q] = (ok && V != nullptr) ? to_f64<TV>(V[row + (int64_t)(j0 + j) * a.ldv]) : 0.0;
    mpre[q] = (ok && a.mask != nullptr) ? a.mask[j0 + j] : 0;
  }
  ACC acc[NR][NN_NB];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int j = 0; j < NN_NB; ++j) acc[r][j] = ACC(0);
  for (int t0 = 0; t0 < m; t0 += NN_ZT) {
    const int tn = (m - t0 < NN_ZT) ? m - t0 : NN_ZT;
    __syncthreads();
    for (int e = tid; e < tn * NN_NB; e += 256) {
      const int i = e / NN_NB, j = e - i * NN_NB;
      double z = (j0 + j < nb) ? a.Z[(int64_t)(t0 + i) * a.ldz + j0 + j] : 0.0;
      if (a.ascale != nullptr) z *= a.ascale[t0 + i];
      zs[e] = (ACC)z;
    }
    __syncthreads();
    for (int i = g; i < tn; i += G * BATCH) {
      RAW raw[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int ii = i + G * u;
        if (ii < tn && rok)
          raw[u] = *(const RAW*)(abase + (int64_t)(t0 + ii) * lda * (int64_t)sizeof(TA));
        else
          raw[u] = RAW{};
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int ii = i + G * u;
        if (ii >= tn) continue;
        ACC av[NR];
        if constexpr (sizeof(TA) == 1) {
          // hardware E4M3 -> float32 conversion (exact), two codes at a time
          const uint32_t ws[2] = {raw[u].x, raw[u].y};
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)ws[q], false);
            const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)ws[q], true);
            av[4 * q + 0] = (ACC)lo.x;
            av[4 * q + 1] = (ACC)lo.y;
            av[4 * q + 2] = (ACC)hi.x;
            av[4 * q + 3] = (ACC)hi.y;
          }
        } else {
          const uint32_t ws[4] = {raw[u].x, raw[u].y, raw[u].z, raw[u].w};
#pragma unroll
          for (int r = 0; r < NR; ++r) {
            const uint32_t h = (ws[r >> 1] >> (16 * (r & 1))) & 0xffffu;
            av[r] = (ACC)__uint_as_float(h << 16);  // bfloat16 -> float, exact
          }
        }
        const ACC* zr = zs + ii * NN_NB;
#pragma unroll
        for (int r = 0; r < NR; ++r)
#pragma unroll
          for (int j = 0; j < NN_NB; ++j) acc[r][j] += av[r] * zr[j];
      }
    }
  }
  // column groups gq = 0..3 of the wave hold the same rows: (0 + 1) + (2 + 3)
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int j = 0; j < NN_NB; ++j) {
      ACC v = acc[r][j];
      v += __shfl_xor(v, 16);
      v += __shfl_xor(v, 32);
      acc[r][j] = v;
    }
  if (gq == 0)
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int j = 0; j < NN_NB; ++j) red[w][8 * rl + r][j] = acc[r][j];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NO; ++q) {
    const int e = tid + 256 * q;
    if (e >= NNN_R * NN_NB) continue;
    const int rr = e % NNN_R, j = e / NNN_R;
    const int64_t row = bx * NNN_R + rr;
    if (row >= d || j0 + j >= nb) continue;
    const ACC sacc = ((red[0][rr][j] + red[1][rr][j]) + red[2][rr][j]) + red[3][rr][j];
    double o = (double)sacc;
    if (alpha != 0.0) o += alpha * vpre[q];
    if (mpre[q] != 0) o = masked_gauss(a.seed, (int64_t)(j0 + j) * d + row);
    const int64_t oi = a.out_row ? row * a.ldo + (j0 + j) : row + (int64_t)(j0 + j) * a.ldo;
    Out[oi] = from_f64<TO>(o);
  }
  __syncthreads();
}

template <typename TA, typename TV, typename TO, typename ACC>
__global__ __launch_bounds__(256) void nn_narrow_kernel(const NnArgs* __restrict__ arr, NnArgs one) {
  const NnArgs a = arr != nullptr ? arr[blockIdx.z] : one;
  if (a.gate != nullptr && *a.gate == 0) return;
  nn_narrow_body<TA, TV, TO, ACC>(a, blockIdx.x, blockIdx.y);
}

// Column-split nn for a narrow A (FP8 or bfloat16), nb <= 8: a workgroup
// owns 512 rows (8 per lane, read with one 8- or 16-byte load per column, so
// a wave instruction moves 512 or 1024 contiguous bytes) and one group of at
// most NNS_KC columns of A; its 4 waves take every fourth column of the
// group, 8 loads in flight each.  Z (scaled by the FP8 column scales) sits in
// LDS as float32; products and sums are float32.  The waves' sums meet in
// LDS in the fixed order (w0 + w1) + (w2 + w3), and each group writes its
// partial rows (8 floats per row) to part + group * d * 8; nn_nsplit_finish
// adds the groups in order, alpha V, and rounds to the output type.
constexpr int NNS_R = 512;
constexpr int NNS_KC = 1024;
template <typename TA>
__global__ __launch_bounds__(256) void nn_nsplit_kernel(int64_t d, int64_t m, int nb,
                                                        const TA* __restrict__ A, int64_t lda,
                                                        const double* __restrict__ Z, int64_t ldz,
                                                        const double* __restrict__ ascale,
                                                        int64_t kc, float* __restrict__ part) {
  constexpr int NR = 8, BATCH = 8, LS = 68;  // LS: LDS floats per lane in the exchange
  typedef uint32_t u32v2 __attribute__((ext_vector_type(2)));
  typedef uint32_t u32v4 __attribute__((ext_vector_type(4)));
  using RAW = typename std::conditional<sizeof(TA) == 1, u32v2, u32v4>::type;
  constexpr int ZN = (NNS_KC * 8 > 2 * 64 * LS) ? NNS_KC * 8 : 2 * 64 * LS;
  __shared__ __attribute__((aligned(16))) float zs[ZN];  // Z, then the exchange
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t c0 = (int64_t)blockIdx.y * kc;
  const int64_t c1 = (c0 + kc < m) ? c0 + kc : m;
  const int tn = (int)(c1 - c0);
  const int64_t row0 = (int64_t)blockIdx.x * NNS_R + 8 * lane;
  for (int e = tid; e < tn * 8; e += 256) {
    const int i = e >> 3, j = e & 7;
    double z = (j < nb) ? Z[(c0 + i) * ldz + j] : 0.0;
    if (ascale != nullptr) z *= ascale[c0 + i];
    zs[e] = (float)z;
  }
  __syncthreads();
  float acc[NR][8];
#pragma unroll
  for (int r = 0; r < NR; ++r)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[r][j] = 0.0f;
  if (row0 < lda) {  // rows d .. lda - 1 of A are zero padding
    const char* abase = (const char*)A + row0 * (int64_t)sizeof(TA);
    for (int i0 = w; i0 < tn; i0 += 4 * BATCH) {
      RAW raw[BATCH];
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int ii = i0 + 4 * u;
        const int ic = ii < tn ? ii : w;  // columns past the group: a valid column, weight 0
        raw[u] = *(const __attribute__((address_space(1))) RAW*)(
            abase + (c0 + ic) * lda * (int64_t)sizeof(TA));
      }
#pragma unroll
      for (int u = 0; u < BATCH; ++u) {
        const int ii = i0 + 4 * u;
        float av[NR];
        if constexpr (sizeof(TA) == 1) {
          const uint32_t ws[2] = {raw[u].x, raw[u].y};
#pragma unroll
          for (int q = 0; q < 2; ++q) {
            const f32x2 lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)ws[q], false);
            const f32x2 hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)ws[q], true);
            av[4 * q + 0] = lo.x;
            av[4 * q + 1] = lo.y;
            av[4 * q + 2] = hi.x;
            av[4 * q + 3] = hi.y;
          }
        } else {
          const uint32_t ws[4] = {raw[u].x, raw[u].y, raw[u].z, raw[u].w};
#pragma unroll
          for (int r = 0; r < NR; ++r)
            av[r] = __uint_as_float(((ws[r >> 1] >> (16 * (r & 1))) & 0xffffu) << 16);
        }
        const float wgt = ii < tn ? 1.0f : 0.0f;
        const f32x4 z0 = *(const f32x4*)(zs + 8 * (ii < tn ? ii : 0));
        const f32x4 z1 = *(const f32x4*)(zs + 8 * (ii < tn ? ii : 0) + 4);
#pragma unroll
        for (int r = 0; r < NR; ++r) {
          const float x = av[r] * wgt;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            acc[r][j] = fmaf(x, z0[j], acc[r][j]);
            acc[r][4 + j] = fmaf(x, z1[j], acc[r][4 + j]);
          }
        }
      }
    }
  }
  // (w0 + w1) + (w2 + w3) through LDS (the Z buffer is free once all waves
  // are past their columns)
  __syncthreads();
  float* xb = zs + (size_t)lane * LS;
  if (w == 1 || w == 3) {
    float* dst = xb + (w == 3 ? 64 * LS : 0);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) dst[8 * r + j] = acc[r][j];
  }
  __syncthreads();
  if (w == 0 || w == 2) {
    const float* src = xb + (w == 2 ? 64 * LS : 0);
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) acc[r][j] += src[8 * r + j];
  }
  __syncthreads();
  if (w == 2)
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
      for (int j = 0; j < 8; ++j) xb[8 * r + j] = acc[r][j];
  __syncthreads();
  if (w == 0) {
    float* out = part + ((int64_t)blockIdx.y * d + row0) * 8;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
      if (row0 + r >= d) break;
      f32x4 o0, o1;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        o0[j] = acc[r][j] + xb[8 * r + j];
        o1[j] = acc[r][4 + j] + xb[8 * r + 4 + j];
      }
      *(f32x4*)(out + 8 * r) = o0;
      *(f32x4*)(out + 8 * r + 4) = o1;
    }
  }
}

// Out(row, j) = alpha V(row, j) + sum over the groups, in group order.
template <typename TV, typename TO>
__global__ __launch_bounds__(256) void nn_nsplit_finish(int64_t d, int nb, int64_t groups,
                                                        const float* __restrict__ part,
                                                        double alpha,
                                                        const double* __restrict__ alpha_p,
                                                        const TV* __restrict__ V, int64_t ldv,
                                                        TO* __restrict__ Out, int64_t ldo) {
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= d) return;
  const double al = (alpha_p != nullptr) ? *alpha_p : alpha;
  double sacc[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) sacc[j] = 0.0;
  for (int64_t g = 0; g < groups; ++g) {
    const f32x4 p0 = *(const f32x4*)(part + (g * d + row) * 8);
    const f32x4 p1 = *(const f32x4*)(part + (g * d + row) * 8 + 4);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sacc[j] += (double)p0[j];
      sacc[4 + j] += (double)p1[j];
    }
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    if (j >= nb) break;
    double o = sacc[j];
    if (al != 0.0 && V != nullptr) o += al * to_f64<TV>(V[row + (int64_t)j * ldv]);
    Out[row + (int64_t)j * ldo] = from_f64<TO>(o);
  }
}

// 64 S rows per wave, 4 waves per workgroup: the tuned value for this
// shape class when there is one, else S = 8 when that still gives 4096
// workgroups (long factors: fewer partial sums), else S = 4 when that still
// gives 1024 workgroups, else 2, else 1 (chosen from the largest entry).
int tn_steps(int64_t d, int64_t m) {
  const int tuned = tune_get(TuneKind::TnSteps, d, m, 0);
  if (tuned == 1 || tuned == 2 || tuned == 4 || tuned == 8) return tuned;
  const int64_t tiles = (m + 15) / 16;
  if (((d + 2047) / 2048) * tiles >= 4096) return 8;
  for (int S : {4, 2}) {
    const int64_t chunks = (d + 256 * S - 1) / (256 * S);
    if (chunks * tiles >= 1024) return S;
  }
  return 1;
}

template <typename TA, typename TB>
hipError_t tn_launch_t(int count, const TnArgs* host, const TnArgs* dev, hipStream_t s) {
  int64_t dmax = 0, mmax = 0, cmax = 0, ymax = 0, zmax = 0;
  for (int p = 0; p < count; ++p) {
    dmax = std::max(dmax, host[p].d);
    mmax = std::max(mmax, host[p].m);
  }
  const int S = tn_steps(dmax, mmax);
  for (int p = 0; p < count; ++p) {
    const TnArgs& a = host[p];
    if (a.d <= 0 || a.m <= 0 || a.nb <= 0) continue;
    if (a.chunks != (a.d + 256 * S - 1) / (256 * S)) return hipErrorInvalidValue;
    cmax = std::max(cmax, a.chunks);
    ymax = std::max(ymax, (a.m + 15) / 16);
    zmax = std::max(zmax, (a.nb + 15) / 16);
  }
  if (cmax == 0) return hipSuccess;
  const TnArgs one = (count == 1) ? host[0] : TnArgs{};
  const TnArgs* arr = (count == 1) ? nullptr : dev;
  if constexpr (sizeof(TA) <= 2 && (std::is_same<TB, float>::value || sizeof(TB) == 2)) {
    // narrow A, float32 or bfloat16 B of at most 8 columns, 16-byte aligned
    // columns: the bfloat16 matrix cores (chunks of whole 32 KB slabs)
    constexpr int SR = 32768 / (64 * (int)sizeof(TA));
    static const bool off = std::getenv("EDA_NARROW_F64") != nullptr;
    bool ok = !off && (256 * S) % SR == 0;
    for (int p = 0; p < count && ok; ++p) {
      const TnArgs& a = host[p];
      ok = a.nb <= 8 && ((a.lda * (int64_t)sizeof(TA)) % 16 == 0) && ((uintptr_t)a.A % 16 == 0) &&
           ((a.ldb * (int64_t)sizeof(TB)) % 16 == 0) && ((uintptr_t)a.B % 16 == 0);
    }
    if (ok) {
      dim3 g((unsigned)cmax, (unsigned)((mmax + 63) / 64), (unsigned)count);
      if (S == 8)
        hipLaunchKernelGGL((tn_narrow_kernel<TA, TB, 8>), g, dim3(256), 0, s, arr, one);
      else if (S == 4)
        hipLaunchKernelGGL((tn_narrow_kernel<TA, TB, 4>), g, dim3(256), 0, s, arr, one);
      else if (S == 2)
        hipLaunchKernelGGL((tn_narrow_kernel<TA, TB, 2>), g, dim3(256), 0, s, arr, one);
      else if constexpr (sizeof(TA) == 2)
        hipLaunchKernelGGL((tn_narrow_kernel<TA, TB, 1>), g, dim3(256), 0, s, arr, one);
      return hipGetLastError();
    }
  }
  if constexpr (sizeof(TA) >= 4) {
    // narrow B, 16-byte aligned columns of A and VW-element aligned columns
    // of B: the streaming kernel with vector loads
    constexpr int VW = 16 / (int)sizeof(TA);
    bool vec = zmax == 1;
    for (int p = 0; p < count && vec; ++p) {
      const TnArgs& a = host[p];
      vec = ((a.lda * (int64_t)sizeof(TA)) % 16 == 0) && ((uintptr_t)a.A % 16 == 0) &&
            (a.ldb % VW == 0) && ((uintptr_t)a.B % (VW * sizeof(TB)) == 0);
    }
    if (vec) {
      dim3 g((unsigned)cmax, (unsigned)ymax, (unsigned)count);
      // EDA_TN_DIRECT=1 selects the direct-load kernel (for comparisons)
      static const bool direct = std::getenv("EDA_TN_DIRECT") != nullptr;
      bool lds = std::is_same<TA, double>::value && std::is_same<TB, double>::value && !direct;
      int64_t nbmax = 0;
      for (int p = 0; p < count && lds; ++p) {
        lds = host[p].nb <= 16 && host[p].ldb % 2 == 0 && ((uintptr_t)host[p].B % 16) == 0;
        nbmax = std::max(nbmax, host[p].nb);
      }
      if (lds) {
        // B staged as 8 columns when every problem has at most 8 (less LDS,
        // more resident workgroups), else as 16
        const bool w16 = nbmax > 8;
#define EDA_TN_LDS(SS)                                                      \
  if (w16)                                                                  \
    hipLaunchKernelGGL((tn_lds_kernel<SS, 16>), g, dim3(256), 0, s, arr, one); \
  else                                                                      \
    hipLaunchKernelGGL((tn_lds_kernel<SS, 8>), g, dim3(256), 0, s, arr, one)
        if (S == 8)
          EDA_TN_LDS(8);
        else if (S == 4)
          EDA_TN_LDS(4);
        else if (S == 2)
          EDA_TN_LDS(2);
        else
          EDA_TN_LDS(1);
#undef EDA_TN_LDS
        return hipGetLastError();
      }
      if (S == 8)
        hipLaunchKernelGGL((tn_stream_kernel<TA, TB, 8>), g, dim3(256), 0, s, arr, one);
      else if (S == 4)
        hipLaunchKernelGGL((tn_stream_kernel<TA, TB, 4>), g, dim3(256), 0, s, arr, one);
      else if (S == 2)
        hipLaunchKernelGGL((tn_stream_kernel<TA, TB, 2>), g, dim3(256), 0, s, arr, one);
      else
        hipLaunchKernelGGL((tn_stream_kernel<TA, TB, 1>), g, dim3(256), 0, s, arr, one);
      return hipGetLastError();
    }
  }
  // column tiles per workgroup: doubled while the grid keeps 1024 workgroups
  // (wide A: B is then read once per CT tiles instead of once per tile)
  int CT = 1;
  // wide B (more than one 16-column tile): three B tiles per workgroup, so
  // that A is read once per 48 columns of B, while that still leaves 1024
  // workgroups
  const int ZT = (zmax >= 2 && cmax * ymax * ((zmax + 2) / 3) * count >= 1024) ? 3 : 1;
  const int64_t zgs = (zmax + ZT - 1) / ZT;
  const int ctmax = (ZT == 1) ? 8 : 2;  // (register budget with three B tiles)
  if (S == 4 && sizeof(TA) == 8)  // (narrow A is bound by its conversions, not by B)
    while (CT < ctmax && cmax * ((ymax + 2 * CT - 1) / (2 * CT)) * zgs * count >= 1024) CT *= 2;
  const int64_t yg = (ymax + CT - 1) / CT;
  const int64_t zg = (zmax + ZT - 1) / ZT;
  dim3 g((unsigned)cmax, (unsigned)(yg * zg), (unsigned)count);
#define TN_GO(S_, CT_) \
  hipLaunchKernelGGL((tn_mfma_kernel<TA, TB, S_, CT_, 1>), g, dim3(256), 0, s, arr, one, (int)yg)
#define TN_GOW(S_) \
  hipLaunchKernelGGL((tn_mfma_kernel<TA, TB, S_, 1, 3>), g, dim3(256), 0, s, arr, one, (int)yg)
  if (ZT == 3) {
    if (S == 8)
      TN_GOW(8);
    else if (S == 4 && CT == 2)
      hipLaunchKernelGGL((tn_mfma_kernel<TA, TB, 4, 2, 3>), g, dim3(256), 0, s, arr, one, (int)yg);
    else if (S == 4)
      TN_GOW(4);
    else if (S == 2)
      TN_GOW(2);
    else
      TN_GOW(1);
  } else if (S == 8) {
    TN_GO(8, 1);
  } else if (S == 4) {
    if (CT == 8)
      TN_GO(4, 8);
    else if (CT == 4)
      TN_GO(4, 4);
    else if (CT == 2)
      TN_GO(4, 2);
    else
      TN_GO(4, 1);
  } else if (S == 2) {
    TN_GO(2, 1);
  } else {
    TN_GO(1, 1);
  }
#undef TN_GO
#undef TN_GOW
  return hipGetLastError();
}

// Rows per nn workgroup: 64 when that still gives 384 workgroups (long
// loops, little Z traffic), else 32, else 16 (more workgroups); chosen from
// the largest entry.  Loads per batch: 16 for small d (few workgroups, so
// one memory round trip per lane matters most), else 4 or 8 (measured
// faster for the streaming passes over P).
template <typename TA, typename TV, typename TO, typename ACC>
hipError_t nn_launch_t(int count, const NnArgs* host, const NnArgs* dev, hipStream_t s) {
  int64_t dmax = 0, ymax = 0, nbmax = 0;
  bool wide_in_place = false;
  for (int p = 0; p < count; ++p) {
    const NnArgs& a = host[p];
    if (a.d <= 0 || a.nb <= 0) continue;
    if (a.m < 0) return hipErrorInvalidValue;
    // In-place Out == A is only safe when one workgroup column covers all
    // nb: up to 8 columns in every kernel, up to 16 in the streaming one.
    if (a.Out == a.A && a.nb > NN_NB) wide_in_place = true;
    dmax = std::max(dmax, a.d);
    ymax = std::max(ymax, (a.nb + NN_NB - 1) / NN_NB);
    nbmax = std::max(nbmax, a.nb);
  }
  if (dmax == 0) return hipSuccess;
  const NnArgs one = (count == 1) ? host[0] : NnArgs{};
  const NnArgs* arr = (count == 1) ? nullptr : dev;
  if constexpr (sizeof(TA) >= 4) {
    // long A with 16-byte aligned columns and at most 16 output columns: the
    // streaming kernel, when it still gets 256
    // workgroups (or the launch is a column-split one or an in-place one of
    // more than 8 columns, which only it implements)
    constexpr int R = 64 * Vec16<TA>::VW;
    constexpr int NBS = 16;
    bool split = false, stream = nbmax <= NBS;
    for (int p = 0; p < count && stream; ++p) {
      const NnArgs& a = host[p];
      split = split || a.kcols > 0;
      stream = ((a.lda * (int64_t)sizeof(TA)) % 16 == 0) && ((uintptr_t)a.A % 16 == 0) &&
               a.ascale == nullptr &&
               (a.Out != a.A || (a.kcols == 0 && a.out_row == 0 && a.ldo == a.lda &&
                                 std::is_same<TO, TA>::value));
    }
    if (split && (!stream || count != 1)) return hipErrorInvalidValue;
    if (wide_in_place && !stream) return hipErrorInvalidValue;
    if (stream && (split || wide_in_place || (dmax + R - 1) / R >= 256)) {
      const int64_t groups = split ? (host[0].m + host[0].kcols - 1) / host[0].kcols : 1;
      const dim3 g((unsigned)((dmax + R - 1) / R), (unsigned)groups, (unsigned)count);
      if (nbmax > NN_NB) {
        hipLaunchKernelGGL((nn_stream_kernel<TA, TV, TO, 16>), g, dim3(256), 0, s, arr, one);
      } else {
        hipLaunchKernelGGL((nn_stream_kernel<TA, TV, TO, 8>), g, dim3(256), 0, s, arr, one);
      }
      return hipGetLastError();
    }
  }
  if (wide_in_place) return hipErrorInvalidValue;
  for (int p = 0; p < count; ++p)
    if (host[p].kcols > 0) return hipErrorInvalidValue;
  if constexpr (sizeof(TA) <= 2) {
    // narrow A with 8-row-aligned columns (the padded storage of P): 8 rows
    // per lane in one load
    bool aligned = true;
    for (int p = 0; p < count; ++p)
      aligned = aligned && host[p].lda % 8 == 0 && ((uintptr_t)host[p].A % 16) == 0;
    if (aligned) {
      hipLaunchKernelGGL((nn_narrow_kernel<TA, TV, TO, ACC>),
                         dim3((unsigned)((dmax + NNN_R - 1) / NNN_R), (unsigned)ymax, (unsigned)count),
                         dim3(256), 0, s, arr, one);
      return hipGetLastError();
    }
  }
  if constexpr (std::is_same<TA, double>::value && std::is_same<TV, double>::value &&
                std::is_same<TO, double>::value) {
    bool plain = nbmax > NN_NB && dmax >= 8192;
    for (int p = 0; p < count && plain; ++p)
      plain = host[p].mask == nullptr && host[p].ascale == nullptr && host[p].out_row == 0 &&
              host[p].Out != host[p].A;
    if (plain && count == 1) {
      // a single wide product with a long inner dimension: the LDS-tiled
      // matrix-core GEMM (64 x 64 output tiles, double-buffered slices)
      const NnArgs& a = host[0];
      const bool al = a.lda % 2 == 0 && ((uintptr_t)a.A % 16) == 0;
      if (al && a.gate == nullptr && a.nb >= 48 && a.m >= 64)
        return launch_gemm_av(a.d, a.nb, a.m, (const double*)a.A, a.lda, a.Z, a.ldz, a.alpha,
                              a.alpha_p, (const double*)a.V, a.ldv, (double*)a.Out, a.ldo, s);
    }
    if (plain) {
      // matrix cores: CTN output tiles per workgroup, as many as leave 512
      // workgroups (A is then read once per 16 CTN columns)
      const int64_t rb = (dmax + 63) / 64;
      int ctn = 8;
      while (ctn > 1 && rb * ((nbmax + 16 * ctn - 1) / (16 * ctn)) * count < 512) ctn /= 2;
      const dim3 g((unsigned)rb, (unsigned)((nbmax + 16 * ctn - 1) / (16 * ctn)), (unsigned)count);
      if (ctn == 8)
        hipLaunchKernelGGL(nn_mfma_kernel<8>, g, dim3(256), 0, s, arr, one);
      else if (ctn == 4)
        hipLaunchKernelGGL(nn_mfma_kernel<4>, g, dim3(256), 0, s, arr, one);
      else if (ctn == 2)
        hipLaunchKernelGGL(nn_mfma_kernel<2>, g, dim3(256), 0, s, arr, one);
      else
        hipLaunchKernelGGL(nn_mfma_kernel<1>, g, dim3(256), 0, s, arr, one);
      return hipGetLastError();
    }
  }
  if (nbmax > NN_NB && dmax >= 8192) {
    // wide outputs over a long A: A streams once per NNW_NB columns (short
    // operands, such as the cores, keep the many small workgroups of the
    // 8-column kernel)
    const unsigned yw = (unsigned)((nbmax + NNW_NB - 1) / NNW_NB);
    if (dmax / 64 >= 256)
      hipLaunchKernelGGL((nn_wide_kernel<TA, TV, TO, ACC, 64, 8>),
                         dim3((unsigned)((dmax + 63) / 64), yw, (unsigned)count), dim3(256), 0, s,
                         arr, one);
    else
      hipLaunchKernelGGL((nn_wide_kernel<TA, TV, TO, ACC, 32, 8>),
                         dim3((unsigned)((dmax + 31) / 32), yw, (unsigned)count), dim3(256), 0, s,
                         arr, one);
    return hipGetLastError();
  }
#define NN_GO(R_, B_)                                                                          \
  hipLaunchKernelGGL((nn_kernel<TA, TV, TO, ACC, R_, B_>),                                     \
                     dim3((unsigned)((dmax + R_ - 1) / R_), (unsigned)ymax, (unsigned)count), \
                     dim3(256), 0, s, arr, one)
  int64_t mmax = 0;
  for (int p = 0; p < count; ++p) mmax = std::max(mmax, host[p].m);
  int cfg = tune_get(TuneKind::NnTile, dmax, mmax, (int)sizeof(TA));
  if (cfg < 0 || cfg >= kNnConfigs)
    cfg = (dmax / 64 >= 384) ? 3 : (dmax / 32 >= 384) ? 2 : (dmax > 4096) ? 0 : 1;
  if (cfg == 3)
    NN_GO(64, 8);
  else if (cfg == 2)
    NN_GO(32, 8);
  else if (cfg == 0)
    NN_GO(16, 4);
  else  // few workgroups (core products): all loads of a lane in one batch
    NN_GO(16, 16);
#undef NN_GO
  return hipGetLastError();
}

}  // namespace

int64_t tn_chunks_for(int64_t d, int64_t dmax, int64_t mmax) {
  const int S = tn_steps(dmax, mmax);
  return (d + 256 * S - 1) / (256 * S);
}

int64_t tn_chunks(int64_t d, int64_t m, int64_t nb) {
  (void)nb;
  return tn_chunks_for(d, d, m);
}

hipError_t launch_tn_multi(int count, const TnArgs* host, const TnArgs* dev, DT adt, DT bdt,
                           hipStream_t s) {
  if (count < 1) return hipSuccess;
  using bf = __hip_bfloat16;
  if (adt == DT::F64 && bdt == DT::F64) return tn_launch_t<double, double>(count, host, dev, s);
  if (adt == DT::F32 && bdt == DT::F32) return tn_launch_t<float, float>(count, host, dev, s);
  if (adt == DT::F32 && bdt == DT::F64) return tn_launch_t<float, double>(count, host, dev, s);
  if (adt == DT::F64 && bdt == DT::F32) return tn_launch_t<double, float>(count, host, dev, s);
  if (adt == DT::BF16 && bdt == DT::F32) return tn_launch_t<bf, float>(count, host, dev, s);
  if (adt == DT::BF16 && bdt == DT::F64) return tn_launch_t<bf, double>(count, host, dev, s);
  if (adt == DT::FP8 && bdt == DT::F32) return tn_launch_t<fp8e4m3, float>(count, host, dev, s);
  if (adt == DT::FP8 && bdt == DT::F64) return tn_launch_t<fp8e4m3, double>(count, host, dev, s);
  if (adt == DT::BF16 && bdt == DT::BF16) return tn_launch_t<bf, bf>(count, host, dev, s);
  if (adt == DT::FP8 && bdt == DT::BF16) return tn_launch_t<fp8e4m3, bf>(count, host, dev, s);
  return hipErrorInvalidValue;
}

hipError_t launch_tn_partial(int64_t d, int64_t m, int64_t nb, const void* A, DT adt,
                             int64_t lda, const void* B, DT bdt, int64_t ldb, double* part,
                             int64_t chunks, const int* gate, hipStream_t s,
                             const double* ascale) {
  if (d <= 0 || m <= 0 || nb <= 0) return hipSuccess;
  TnArgs a{d, m, nb, lda, ldb, chunks, A, B, part, gate, ascale};
  return launch_tn_multi(1, &a, nullptr, adt, bdt, s);
}

hipError_t launch_reduce_multi(int count, const ReduceArgs* host, const ReduceArgs* dev,
                               hipStream_t s) {
  int64_t xmax = 0;
  for (int p = 0; p < count; ++p) xmax = std::max(xmax, (host[p].m * host[p].nb + 63) / 64);
  if (xmax == 0) return hipSuccess;
  const ReduceArgs one = (count == 1) ? host[0] : ReduceArgs{};
  const ReduceArgs* arr = (count == 1) ? nullptr : dev;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)xmax, 1, (unsigned)count), dim3(256),
                     0, s, arr, one);
  return hipGetLastError();
}

hipError_t launch_reduce_partials(int64_t chunks, int64_t m, int64_t nb, const double* part,
                                  double alpha, double beta, double* C_col, int64_t ldc,
                                  double zalpha, double* Z_row, int64_t ldz, const int* gate,
                                  hipStream_t s, int64_t mc, double* C2, int64_t ldc2) {
  if (m * nb <= 0) return hipSuccess;
  if (mc >= 0 && C2 == nullptr) return hipErrorInvalidValue;
  ReduceArgs a{chunks, m, nb, ldc, ldz, part, alpha, beta, zalpha, C_col, Z_row, gate};
  a.mc = mc;
  a.C2 = C2;
  a.ldc2 = ldc2;
  return launch_reduce_multi(1, &a, nullptr, s);
}

hipError_t launch_nn_multi(int count, const NnArgs* host, const NnArgs* dev, DT adt, DT vdt,
                           DT odt, hipStream_t s) {
  if (count < 1) return hipSuccess;
  using bf = __hip_bfloat16;
#define NN_CASE(a, v, o, TA, TV, TO, ACC)                                    \
  if (adt == DT::a && vdt == DT::v && odt == DT::o)                          \
    return nn_launch_t<TA, TV, TO, ACC>(count, host, dev, s);
  NN_CASE(F64, F64, F64, double, double, double, double)
  NN_CASE(F32, F32, F32, float, float, float, float)
  NN_CASE(F32, F64, F64, float, double, double, double)
  NN_CASE(F64, F64, F32, double, double, float, double)
  NN_CASE(F64, F32, F32, double, float, float, double)
  NN_CASE(BF16, F32, F32, bf, float, float, float)
  NN_CASE(BF16, F64, F64, bf, double, double, double)
  NN_CASE(FP8, F32, F32, fp8e4m3, float, float, float)
  NN_CASE(FP8, F64, F64, fp8e4m3, double, double, double)
  NN_CASE(BF16, BF16, BF16, bf, bf, bf, float)
  NN_CASE(FP8, BF16, BF16, fp8e4m3, bf, bf, float)
#undef NN_CASE
  return hipErrorInvalidValue;
}

int64_t nn_split_groups(int64_t m) {
  // 128-row workgroups; column groups of at least 64 columns, as many as
  // give about 512 workgroups
  const int64_t rb = (m + 127) / 128;
  int64_t g = (512 + rb - 1) / rb;
  g = std::max<int64_t>(1, std::min(g, (m + 63) / 64));
  const int64_t kc = (m + g - 1) / g;
  return (m + kc - 1) / kc;
}

int64_t nn_narrow_split_groups(int64_t d, int64_t m) {
  // about 512 workgroups, column groups of at least 64 and at most NNS_KC
  // (the pass is bound by its float32 FMAs, 8 per factor entry, so more
  // groups only add partial rows)
  const int64_t rb = (d + NNS_R - 1) / NNS_R;
  int64_t g = (512 + rb - 1) / rb;
  g = std::max<int64_t>(g, (m + NNS_KC - 1) / NNS_KC);
  g = std::min<int64_t>(g, std::max<int64_t>(1, (m + 63) / 64));
  g = std::max<int64_t>(g, (m + NNS_KC - 1) / NNS_KC);
  const int64_t kc = (m + g - 1) / g;
  return (m + kc - 1) / kc;
}

hipError_t launch_nn_narrow_split(int64_t d, int64_t m, int64_t nb, const void* A, DT adt,
                                  int64_t lda, const double* Z, int64_t ldz, double alpha,
                                  const double* alpha_p, const void* V, DT vdt, int64_t ldv,
                                  void* Out, DT odt, int64_t ldo, const double* ascale,
                                  float* part, hipStream_t s) {
  if (d <= 0 || nb <= 0) return hipSuccess;
  if (m <= 0 || nb > 8 || (adt != DT::BF16 && adt != DT::FP8) || vdt != odt || vdt == DT::F64 ||
      (lda % 8) != 0 || ((uintptr_t)A % 16) != 0 || ((uintptr_t)part % 16) != 0)
    return hipErrorInvalidValue;
  const int64_t groups = nn_narrow_split_groups(d, m);
  const int64_t kc = (m + groups - 1) / groups;
  if (kc > NNS_KC) return hipErrorInvalidValue;
  const dim3 g((unsigned)((d + NNS_R - 1) / NNS_R), (unsigned)groups);
  if (adt == DT::FP8)
    hipLaunchKernelGGL(nn_nsplit_kernel<fp8e4m3>, g, dim3(256), 0, s, d, m, (int)nb,
                       (const fp8e4m3*)A, lda, Z, ldz, ascale, kc, part);
  else
    hipLaunchKernelGGL(nn_nsplit_kernel<__hip_bfloat16>, g, dim3(256), 0, s, d, m, (int)nb,
                       (const __hip_bfloat16*)A, lda, Z, ldz, ascale, kc, part);
  const dim3 gf((unsigned)((d + 255) / 256));
  using bf = __hip_bfloat16;
  if (odt == DT::F32)
    hipLaunchKernelGGL((nn_nsplit_finish<float, float>), gf, dim3(256), 0, s, d, (int)nb, groups,
                       part, alpha, alpha_p, (const float*)V, ldv, (float*)Out, ldo);
  else if (odt == DT::BF16)
    hipLaunchKernelGGL((nn_nsplit_finish<bf, bf>), gf, dim3(256), 0, s, d, (int)nb, groups, part,
                       alpha, alpha_p, (const bf*)V, ldv, (bf*)Out, ldo);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_nn_split(int64_t m, int64_t nb, const double* C, int64_t ldc, const double* Y,
                           int64_t ldy, double* part, double* Z, int64_t ldz, hipStream_t s) {
  if (m <= 0 || nb <= 0) return hipSuccess;
  if (nb > 16 || (ldc * 8) % 16 != 0 || (uintptr_t)C % 16 != 0) return hipErrorInvalidValue;
  const int64_t groups = nn_split_groups(m);
  const int64_t kc = (m + groups - 1) / groups;
  NnArgs a{m, m, nb, ldc, ldy, 0, nb, C, Y, 0.0, nullptr, part, 1, nullptr, nullptr, nullptr,
           nullptr, 0};
  a.kcols = kc;
  hipError_t e = nn_launch_t<double, double, double, double>(1, &a, nullptr, s);
  if (e != hipSuccess) return e;
  return launch_reduce_partials(groups, m, nb, part, 0.0, 0.0, nullptr, 0, 1.0, Z, ldz, nullptr, s);
}

hipError_t launch_nn(int64_t d, int64_t m, int64_t nb, const void* A, DT adt, int64_t lda,
                     const double* Z, int64_t ldz, double alpha, const void* V, DT vdt,
                     int64_t ldv, void* Out, DT odt, int64_t ldo, const int* gate,
                     hipStream_t s, bool out_row, const double* alpha_p,
                     const double* ascale, const int* mask, uint64_t seed) {
  if (d <= 0 || nb <= 0) return hipSuccess;
  NnArgs a{d, m, nb, lda, ldz, ldv, ldo, A, Z, alpha, V, Out, out_row ? 1 : 0, gate, alpha_p,
           ascale, mask, seed};
  return launch_nn_multi(1, &a, nullptr, adt, vdt, odt, s);
}

}  // namespace eda
