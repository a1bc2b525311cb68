// Nearest-neighbour classification in the EDA subspace (Section 3.3): the
// distance between a training sample x_i and a testing sample y_j is
// ||X^T (x_i - y_j)||_2 for the orthonormal d x t result X of eda_solve, and
// a testing sample takes the label of its nearest training sample (1-NN).
// The projections X^T x_i and X^T y_j are the chunked transposed products of
// the solver (matrix cores, fixed-order reduction), the pairwise distances
// and the arg-min one workgroup per testing sample.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "host_internal.h"

using namespace eda;

namespace {

// Row-major projections (n x t) of the n columns of S (d x n, lds) onto X.
eda_status project(eda_handle h, int64_t d, int64_t t, const double* X, int64_t ldx, int64_t n,
                   const double* S, int64_t lds, Buf& out) {
  const int64_t chunks = tn_chunks(d, n, t);
  STCHK(ensure(h, h->part, (size_t)chunks * n * t * 8));
  STCHK(ensure(h, out, (size_t)n * t * 8));
  HIPCHK(launch_tn_partial(d, n, t, S, DT::F64, lds, X, DT::F64, ldx, h->part.d(), chunks,
                           nullptr, h->stream));
  HIPCHK(launch_reduce_partials(chunks, n, t, h->part.d(), 0.0, 0.0, nullptr, 0, 1.0, out.d(), t,
                                nullptr, h->stream));
  return EDA_OK;
}

}  // namespace

extern "C" eda_status eda_nn_classify(eda_handle h, int64_t d, int64_t t, const double* X,
                                      int64_t ldx, int64_t n_train, const double* train,
                                      int64_t ldtr, const int32_t* train_labels, int64_t n_test,
                                      const double* test, int64_t ldte, int32_t* pred,
                                      int64_t* nn_index, double* nn_dist) {
  if (h == nullptr) return EDA_ERR_ARG;
  if (d < 1 || t < 1 || t > 1024 || t > d)
    return fail(h, EDA_ERR_ARG, "need 1 <= t <= min(d, 1024), got d=%lld t=%lld", (long long)d,
                (long long)t);
  if (n_train < 1 || n_test < 1) return fail(h, EDA_ERR_ARG, "need n_train >= 1 and n_test >= 1");
  if (n_test > INT32_MAX) return fail(h, EDA_ERR_ARG, "n_test exceeds 2^31 - 1");
  if (ldx < d || ldtr < d || ldte < d) return fail(h, EDA_ERR_ARG, "leading dimensions must be >= d");
  if (X == nullptr || train == nullptr || train_labels == nullptr || test == nullptr ||
      pred == nullptr || nn_index == nullptr || nn_dist == nullptr)
    return fail(h, EDA_ERR_ARG, "null pointer");
  STCHK(need_device(h));
  STCHK(check_dev_ptr(h, X, "X"));
  STCHK(check_dev_ptr(h, train, "train"));
  STCHK(check_dev_ptr(h, train_labels, "train_labels"));
  STCHK(check_dev_ptr(h, test, "test"));
  STCHK(check_dev_ptr(h, pred, "pred"));
  STCHK(check_dev_ptr(h, nn_index, "nn_index"));
  STCHK(check_dev_ptr(h, nn_dist, "nn_dist"));
  STCHK(project(h, d, t, X, ldx, n_train, train, ldtr, h->nnp[0]));
  STCHK(project(h, d, t, X, ldx, n_test, test, ldte, h->nnp[1]));
  HIPCHK(launch_nn_classify(n_train, n_test, t, h->nnp[0].d(), h->nnp[1].d(), train_labels, pred,
                            nn_index, nn_dist, h->stream));
  return EDA_OK;
}
