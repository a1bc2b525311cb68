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
// for nb = 8 every element of A feeds 8 FMAs, far below the FP64 ridge.
//
// tn mapping: a 256-thread workgroup owns a chunk of rows and 32 columns of A
// (8 per wave); lanes own rows, so every load of a column is a contiguous
// 512-byte wave access.  Each lane keeps an 8 x 8 tile of partial dot
// products in registers and the wave folds the 64 values over its 64 lanes
// with a butterfly reduce-scatter (63 shuffles), after which lane l holds
// entry l of the tile.
//
// nn mapping: a workgroup owns 64 rows; its 4 waves split the m columns of A
// and the wave partials are summed in a fixed order through LDS.  Z is read
// with wave-uniform addresses (scalar loads / broadcast).
#include "common.h"

namespace eda {

namespace {

constexpr int TN_MT = 8;   // A columns per wave
constexpr int TN_NB = 8;   // B columns per tile
constexpr int NN_NB = 8;   // output columns per workgroup

// Butterfly reduce-scatter of 64 values across the 64 lanes of a wave: on
// return lane l holds sum over lanes of v[l].
template <typename T>
__device__ __forceinline__ T wave_reduce_scatter64(T (&v)[64], int lane) {
#pragma unroll
  for (int h = 32; h >= 1; h >>= 1) {
    const bool up = (lane & h) != 0;
#pragma unroll
    for (int i = 0; i < h; ++i) {
      const T send = up ? v[i] : v[i + h];
      const T keep = up ? v[i + h] : v[i];
      v[i] = keep + __shfl_xor(send, h);
    }
  }
  return v[0];
}

template <typename TA, typename TB, typename ACC>
__global__ __launch_bounds__(256) void tn_partial_kernel(int64_t d, int m, int nb,
                                                         const TA* __restrict__ A, int64_t lda,
                                                         const TB* __restrict__ B, int64_t ldb,
                                                         double* __restrict__ part,
                                                         int64_t rows_per_chunk,
                                                         const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t chunk = blockIdx.x;
  const int i0 = (blockIdx.y * 4 + wid) * TN_MT;
  const int j0 = blockIdx.z * TN_NB;
  const int64_t r0 = chunk * rows_per_chunk;
  const int64_t r1 = (r0 + rows_per_chunk < d) ? r0 + rows_per_chunk : d;

  ACC acc[TN_MT][TN_NB];
#pragma unroll
  for (int i = 0; i < TN_MT; ++i)
#pragma unroll
    for (int j = 0; j < TN_NB; ++j) acc[i][j] = ACC(0);

  if (i0 < m) {
    const TA* ap[TN_MT];
    const TB* bp[TN_NB];
    bool aok[TN_MT], bok[TN_NB];
#pragma unroll
    for (int i = 0; i < TN_MT; ++i) {
      aok[i] = (i0 + i) < m;
      ap[i] = A + (int64_t)(aok[i] ? i0 + i : i0) * lda;
    }
#pragma unroll
    for (int j = 0; j < TN_NB; ++j) {
      bok[j] = (j0 + j) < nb;
      bp[j] = B + (int64_t)(bok[j] ? j0 + j : j0) * ldb;
    }
#pragma unroll 2
    for (int64_t r = r0 + lane; r < r1; r += 64) {
      ACC av[TN_MT], bv[TN_NB];
#pragma unroll
      for (int i = 0; i < TN_MT; ++i) av[i] = aok[i] ? to_acc<ACC>(ap[i][r]) : ACC(0);
#pragma unroll
      for (int j = 0; j < TN_NB; ++j) bv[j] = bok[j] ? to_acc<ACC>(bp[j][r]) : ACC(0);
#pragma unroll
      for (int i = 0; i < TN_MT; ++i)
#pragma unroll
        for (int j = 0; j < TN_NB; ++j) acc[i][j] += av[i] * bv[j];
    }
  }

  ACC v[64];
#pragma unroll
  for (int e = 0; e < 64; ++e) v[e] = acc[e / TN_NB][e % TN_NB];
  const ACC tot = wave_reduce_scatter64<ACC>(v, lane);
  const int i = lane / TN_NB, j = lane % TN_NB;
  if (i0 + i < m && j0 + j < nb)
    part[(chunk * m + (i0 + i)) * (int64_t)nb + (j0 + j)] = (double)tot;
}

__global__ __launch_bounds__(256) void reduce_partials_kernel(int64_t chunks, int64_t m, int64_t nb,
                                                              const double* __restrict__ part,
                                                              double alpha, double beta,
                                                              double* __restrict__ C, int64_t ldc,
                                                              double zalpha, double* __restrict__ Z,
                                                              int64_t ldz, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t mn = m * nb;
  if (e >= mn) return;
  // fixed order; eight independent loads in flight per thread
  double s = 0.0;
  int64_t c = 0;
  for (; c + 8 <= chunks; c += 8) {
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = part[(c + q) * mn + e];
#pragma unroll
    for (int q = 0; q < 8; ++q) s += v[q];
  }
  for (; c < chunks; ++c) s += part[c * mn + e];
  const int64_t i = e / nb, j = e - i * nb;
  if (C != nullptr) {
    double* cp = C + i + j * ldc;
    *cp = (beta == 0.0 ? 0.0 : beta * *cp) + alpha * s;
  }
  if (Z != nullptr) Z[i * ldz + j] = zalpha * s;
}

template <typename TA, typename TV, typename TO, typename ACC>
__global__ __launch_bounds__(256) void nn_kernel(int64_t d, int m, int nb, const TA* __restrict__ A,
                                                 int64_t lda, const double* __restrict__ Z,
                                                 int64_t ldz, double alpha, const TV* __restrict__ V,
                                                 int64_t ldv, TO* __restrict__ Out, int64_t ldo,
                                                 int out_row, const int* __restrict__ gate) {
  if (gate != nullptr && *gate == 0) return;
  __shared__ ACC red[3][64][NN_NB + 1];
  const int lane = threadIdx.x & 63;
  const int wid = threadIdx.x >> 6;
  const int64_t r = blockIdx.x * (int64_t)64 + lane;
  const int j0 = blockIdx.y * NN_NB;
  const int mq = (m + 3) / 4;
  const int ib = wid * mq;
  const int ie = (ib + mq < m) ? ib + mq : m;

  ACC acc[NN_NB];
#pragma unroll
  for (int j = 0; j < NN_NB; ++j) acc[j] = ACC(0);
  bool jok[NN_NB];
#pragma unroll
  for (int j = 0; j < NN_NB; ++j) jok[j] = (j0 + j) < nb;

  if (r < d) {
    const TA* ar = A + r;
#pragma unroll 4
    for (int i = ib; i < ie; ++i) {
      const ACC a = to_acc<ACC>(ar[(int64_t)i * lda]);
      const double* zr = Z + (int64_t)i * ldz + j0;
#pragma unroll
      for (int j = 0; j < NN_NB; ++j)
        if (jok[j]) acc[j] += a * (ACC)zr[j];
    }
  }
  if (wid > 0) {
#pragma unroll
    for (int j = 0; j < NN_NB; ++j) red[wid - 1][lane][j] = acc[j];
  }
  __syncthreads();
  if (wid == 0 && r < d) {
#pragma unroll
    for (int w = 0; w < 3; ++w)
#pragma unroll
      for (int j = 0; j < NN_NB; ++j) acc[j] += red[w][lane][j];
#pragma unroll
    for (int j = 0; j < NN_NB; ++j) {
      if (!jok[j]) continue;
      double o = (double)acc[j];
      if (alpha != 0.0) o += alpha * to_f64<TV>(V[r + (int64_t)(j0 + j) * ldv]);
      const int64_t oi = out_row ? r * ldo + (j0 + j) : r + (int64_t)(j0 + j) * ldo;
      Out[oi] = from_f64<TO>(o);
    }
  }
}

void tn_geometry(int64_t d, int64_t m, int64_t nb, int64_t* chunks, int64_t* rows) {
  const int64_t ygroups = ((m + 4 * TN_MT - 1) / (4 * TN_MT)) * ((nb + TN_NB - 1) / TN_NB);
  const int64_t target = 2048;
  int64_t c = (target + ygroups - 1) / ygroups;
  const int64_t cmax = std::max<int64_t>(1, (d + 255) / 256);  // >= 4 rows per lane
  c = std::max<int64_t>(1, std::min(c, cmax));
  int64_t rp = (d + c - 1) / c;
  rp = ((rp + 63) / 64) * 64;
  *rows = rp;
  *chunks = (d + rp - 1) / rp;
}

template <typename TA, typename TB, typename ACC>
hipError_t tn_launch_t(int64_t d, int64_t m, int64_t nb, const void* A, int64_t lda,
                       const void* B, int64_t ldb, double* part, int64_t chunks,
                       const int* gate, hipStream_t s) {
  int64_t c, rows;
  tn_geometry(d, m, nb, &c, &rows);
  if (c != chunks) return hipErrorInvalidValue;
  dim3 g((unsigned)chunks, (unsigned)((m + 4 * TN_MT - 1) / (4 * TN_MT)),
         (unsigned)((nb + TN_NB - 1) / TN_NB));
  hipLaunchKernelGGL((tn_partial_kernel<TA, TB, ACC>), g, dim3(256), 0, s, d, (int)m, (int)nb,
                     (const TA*)A, lda, (const TB*)B, ldb, part, rows, gate);
  return hipGetLastError();
}

template <typename TA, typename TV, typename TO, typename ACC>
hipError_t nn_launch_t(int64_t d, int64_t m, int64_t nb, const void* A, int64_t lda,
                       const double* Z, int64_t ldz, double alpha, const void* V, int64_t ldv,
                       void* Out, int64_t ldo, bool out_row, const int* gate, hipStream_t s) {
  dim3 g((unsigned)((d + 63) / 64), (unsigned)((nb + NN_NB - 1) / NN_NB));
  hipLaunchKernelGGL((nn_kernel<TA, TV, TO, ACC>), g, dim3(256), 0, s, d, (int)m, (int)nb,
                     (const TA*)A, lda, Z, ldz, alpha, (const TV*)V, ldv, (TO*)Out, ldo,
                     out_row ? 1 : 0, gate);
  return hipGetLastError();
}

}  // namespace

int64_t tn_chunks(int64_t d, int64_t m, int64_t nb) {
  int64_t c, rows;
  tn_geometry(d, m, nb, &c, &rows);
  return c;
}

hipError_t launch_tn_partial(int64_t d, int64_t m, int64_t nb, const void* A, DT adt,
                             int64_t lda, const void* B, DT bdt, int64_t ldb, double* part,
                             int64_t chunks, const int* gate, hipStream_t s) {
  if (d <= 0 || m <= 0 || nb <= 0) return hipSuccess;
  using bf = __hip_bfloat16;
  if (adt == DT::F64 && bdt == DT::F64)
    return tn_launch_t<double, double, double>(d, m, nb, A, lda, B, ldb, part, chunks, gate, s);
  if (adt == DT::F32 && bdt == DT::F32)
    return tn_launch_t<float, float, float>(d, m, nb, A, lda, B, ldb, part, chunks, gate, s);
  if (adt == DT::F32 && bdt == DT::F64)
    return tn_launch_t<float, double, double>(d, m, nb, A, lda, B, ldb, part, chunks, gate, s);
  if (adt == DT::F64 && bdt == DT::F32)
    return tn_launch_t<double, float, double>(d, m, nb, A, lda, B, ldb, part, chunks, gate, s);
  if (adt == DT::BF16 && bdt == DT::F32)
    return tn_launch_t<bf, float, float>(d, m, nb, A, lda, B, ldb, part, chunks, gate, s);
  if (adt == DT::BF16 && bdt == DT::F64)
    return tn_launch_t<bf, double, double>(d, m, nb, A, lda, B, ldb, part, chunks, gate, s);
  return hipErrorInvalidValue;
}

hipError_t launch_reduce_partials(int64_t chunks, int64_t m, int64_t nb, const double* part,
                                  double alpha, double beta, double* C_col, int64_t ldc,
                                  double zalpha, double* Z_row, int64_t ldz, const int* gate,
                                  hipStream_t s) {
  const int64_t mn = m * nb;
  if (mn <= 0) return hipSuccess;
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)((mn + 255) / 256)), dim3(256), 0, s,
                     chunks, m, nb, part, alpha, beta, C_col, ldc, zalpha, Z_row, ldz, gate);
  return hipGetLastError();
}

hipError_t launch_nn(int64_t d, int64_t m, int64_t nb, const void* A, DT adt, int64_t lda,
                     const double* Z, int64_t ldz, double alpha, const void* V, DT vdt,
                     int64_t ldv, void* Out, DT odt, int64_t ldo, const int* gate,
                     hipStream_t s, bool out_row) {
  if (d <= 0 || nb <= 0) return hipSuccess;
  // In-place Out == A is only safe when one workgroup column covers all nb.
  if (Out == A && nb > NN_NB) return hipErrorInvalidValue;
  using bf = __hip_bfloat16;
#define NN_CASE(a, v, o, TA, TV, TO, ACC)                                                     \
  if (adt == DT::a && vdt == DT::v && odt == DT::o)                                           \
    return nn_launch_t<TA, TV, TO, ACC>(d, m, nb, A, lda, Z, ldz, alpha, V, ldv, Out, ldo,    \
                                        out_row, gate, s);
  NN_CASE(F64, F64, F64, double, double, double, double)
  NN_CASE(F32, F32, F32, float, float, float, float)
  NN_CASE(F32, F64, F64, float, double, double, double)
  NN_CASE(F64, F64, F32, double, double, float, double)
  NN_CASE(F64, F32, F32, double, float, float, double)
  NN_CASE(BF16, F32, F32, bf, float, float, float)
  NN_CASE(BF16, F64, F64, bf, double, double, double)
#undef NN_CASE
  return hipErrorInvalidValue;
}

}  // namespace eda
