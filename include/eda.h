/*
 * eda.h -- C ABI of libeda, the MI355X (gfx950) library for the hot path of
 * inexact-Krylov exponential discriminant analysis (EDA).
 *
 * Problem (Wu, Feng, Zhang, Yang, arXiv 1512.06500, Section 1, eq. (1.7)):
 * find the t dominant eigenpairs of the symmetric-definite pencil
 *
 *     exp(S_B) x = lambda exp(S_W) x,   S_W = H_W H_W^T,  S_B = H_B H_B^T,
 *
 * with H_W (d x n) and H_B (d x k) the within- and between-class scatter
 * factors of eqs. (1.1)-(1.2), and return the eigenvectors orthonormalised in
 * decreasing-lambda order (Algorithm 1 step 4, Algorithm 3 step 6).
 *
 * The library never forms a d x d matrix.  Every exponential is applied as
 *     exp(c H H^T) V = V + H phi_c(H^T H) H^T V,  phi_c(z) = (e^{cz}-1)/z,
 * which equals the closed form of Theorem 3.1 (eqs. (3.9)-(3.11)) and needs
 * only the small Gram matrix H^T H and its symmetric eigendecomposition.
 * The eigenproblem is solved by block Lanczos on the symmetric form
 * M = exp(-S_W/2) exp(S_B) exp(-S_W/2) (eq. (3.15)), then x = exp(-S_W/2) y
 * (eq. (3.14)), as in Algorithm 3.
 *
 * Conventions for every call:
 *   - Matrices are column-major with an explicit leading dimension (ld >= rows).
 *   - Pointers documented as "device" must point to GPU memory of the device
 *     that was current when the handle was created; "host" pointers to CPU
 *     memory.  The caller owns every buffer it passes; the library copies
 *     what it keeps.
 *   - Work is ordered on the handle's HIP stream.  Calls returning host
 *     outputs synchronise that stream before returning; the others do not.
 *   - A handle is not thread-safe; distinct handles are independent.
 *   - Errors are reported by return code only.  Arguments are validated on
 *     the host before any HIP call, so invalid arguments never reach a
 *     kernel.  eda_last_error() gives a message for the last failure.
 */
#ifndef EDA_H_
#define EDA_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct eda_handle_s* eda_handle;

typedef enum {
  EDA_OK = 0,
  EDA_ERR_ARG = 1,        /* invalid argument (shape, ld, null pointer, option)   */
  EDA_ERR_NOMEM = 2,      /* device or host allocation failed                      */
  EDA_ERR_HIP = 3,        /* a HIP runtime call failed                             */
  EDA_ERR_NOCONV = 4,     /* eda_solve: max_iter reached; best pairs still written */
  EDA_ERR_RANGE = 5,      /* a result is outside the floating-point range          */
  EDA_ERR_NONFINITE = 6,  /* NaN or Inf found in an input factor                   */
  EDA_ERR_STATE = 7       /* call order violated (e.g. eda_solve before prepare)  */
} eda_status;

/* Storage / arithmetic types. */
typedef enum { EDA_F64 = 0, EDA_F32 = 1, EDA_BF16 = 2, EDA_FP8_E4M3 = 3 } eda_dtype;

/* Which scatter factor an exponential acts on. */
typedef enum { EDA_W = 0, EDA_B = 1 } eda_which;

/* Operator forms of Section 3.1. */
typedef enum {
  EDA_FORM_LANCZOS_M = 0,  /* M = exp(-S_W/2) exp(S_B) exp(-S_W/2), eq. (3.15), product (3.16) */
  EDA_FORM_ARNOLDI_A = 1,  /* A = exp(-S_W) exp(S_B), eq. (3.1), product (3.2)                 */
  EDA_FORM_JD_M = 2        /* M of eq. (3.15) solved by block Jacobi-Davidson (Section 5)       */
} eda_form;

/* Residual measure used by the stopping test of eda_solve. */
typedef enum {
  EDA_RES_REL_THETA = 0,   /* ||M y - theta y|| / theta per Ritz pair (default) */
  EDA_RES_NORMWISE = 1     /* ||M y - theta y|| / theta_1                        */
} eda_resmode;

/* Solver options.  A zero-initialised struct selects every default. */
typedef struct {
  eda_form form;            /* EDA_FORM_LANCZOS_M (default), EDA_FORM_ARNOLDI_A or
                               EDA_FORM_JD_M                                         */
  int32_t block;            /* block width b (default 8): 1 .. 16 for the Lanczos
                               form, 1 .. 8 for the Arnoldi and Jacobi-Davidson
                               forms and for eda_solve_batched                       */
  int32_t max_basis;        /* basis columns before a thick restart (default
                               max(2t+2b, t+6b) rounded up to a multiple of b,
                               capped by d)                                          */
  int32_t max_iter;         /* maximal block steps (default 4000)                    */
  eda_resmode resmode;
  eda_dtype krylov_dtype;   /* basis type of the Krylov phase: EDA_F64 (default) or
                               EDA_F32.  The operator of that phase uses the storage
                               type given to eda_prepare.                            */
  eda_dtype refine_dtype;   /* arithmetic of the refinement stage; must be EDA_F64   */
  uint64_t seed;            /* start-block seed when start_block is NULL             */
  const void* start_block;  /* device, d x b float64 start block, or NULL            */
  int64_t ld_start;         /* leading dimension of start_block                      */
  int32_t check_every;      /* block steps between Rayleigh-Ritz checks; 0 (default):
                               scheduled from the observed convergence rate        */
  int32_t max_refine;       /* float64 refinement passes after the Krylov phase:
                               0 = default (16 after a phase with a narrower operator
                               or basis, 2 after a float64 one); < 0 = none, and the
                               Krylov-phase pairs are returned with float64 residuals */
  int32_t reserved[6];
} eda_solve_opts;

/* Per-solve diagnostics. */
typedef struct {
  int32_t iters;            /* block Lanczos steps taken                      */
  int32_t restarts;         /* thick restarts                                 */
  int32_t refine_passes;    /* FP64 refinement passes                         */
  int32_t flags;            /* EDA_WARN_* bits                                */
  int64_t ops;              /* operator applications, counted per column      */
  double bytes_moved;       /* algorithmic HBM bytes of the operator passes   */
  double t_prepare_ms;      /* time of the last eda_prepare                   */
  double t_krylov_ms;       /* Krylov phase of this solve                     */
  double t_refine_ms;       /* refinement phase of this solve                 */
  double shift_s;           /* spectral shift s: the operator iterated is e^{-s} M */
  int64_t op_calls;         /* block operator products M V timed in this solve */
  double t_op_ms;           /* their total duration (HIP events on the handle's
                               stream around each product: both streaming
                               passes over P and the small core product)     */
  double op_bytes;          /* algorithmic bytes of one timed product:
                               2 d (n+k) s_P + 3 d b 8 (s_P: bytes per entry) */
} eda_info;

#define EDA_WARN_DEGENERATE 1  /* t > k-1: the wanted subspace is not unique       */
#define EDA_WARN_FLOOR 2       /* some pair stopped at its attainable floor, not tol */
#define EDA_WARN_REPAIRED 4    /* a Krylov block lost rank and was re-orthogonalised */
#define EDA_WARN_FALLBACK 8    /* batched, narrow precision: the refinement stalled and the
                                  problem continued as a float64 block Lanczos solve
                                  started from its refined Ritz block                  */

/* Create a handle bound to the current HIP device and to `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  *h receives the handle. */
eda_status eda_create(eda_handle* h, void* hip_stream);

/* Release every device allocation of the handle and the handle itself.
 * Synchronises the handle's stream first.  NULL is ignored. */
void eda_destroy(eda_handle h);

/* Message for a status code (static string). */
const char* eda_strerror(eda_status s);

/* Message for the last failed call on `h` (valid until the next call). */
const char* eda_last_error(eda_handle h);

/* Scatter factors of eqs. (1.1)-(1.2).
 * X: device, d x n float64, ld ldx >= d, samples as columns, classes stored
 *    contiguously (class j occupies counts[j] consecutive columns).
 * counts: host, k entries (1 <= k <= 65535), each >= 1, summing to n.
 * H_W: device out, d x n (ld ldw >= d): X_j - mu_j e^T per class.
 * H_B: device out, d x k (ld ldb >= d): sqrt(n_j) (mu_j - mu), mu the mean of
 *      all n samples.  Stream-ordered, no synchronisation. */
eda_status eda_scatter_factors(eda_handle h, int64_t d, int64_t n, int64_t k,
                               const double* X, int64_t ldx, const int64_t* counts,
                               double* H_W, int64_t ldw, double* H_B, int64_t ldb);

/* Preprocessing of Algorithm 2 (steps 1-4), in Gram form.
 * H_W: device, d x n float64 (ldw >= d); H_B: device, d x k float64 (ldb >= d).
 * Requires d >= 2, 2 <= k <= n <= 2048.  The factors are copied into library
 * storage P = [H_W H_B] in `storage` precision (EDA_F64, EDA_F32, EDA_BF16, or
 * EDA_FP8_E4M3 with one float64 scale per column: column j is stored as
 * E4M3(P(:, j) / s_j), s_j = max |P(:, j)| / 448; a narrower storage also
 * keeps a float64 master copy, used for the Gram matrix, the refinement
 * stage of eda_solve and the back-transform),
 * the Gram matrix P^T P is formed in float64, eig(H_B^T H_B) (and, when
 * requested, eig(H_W^T H_W)) are computed in float64, and the cores of the
 * exponentials are built.
 * Returns EDA_ERR_NONFINITE if a factor holds NaN/Inf.  H_W and H_B are
 * copied and checked before it returns (they may be reused at once); the
 * cores are then built on the handle's stream without the host waiting, and
 * every later call on the handle is ordered after them. */
eda_status eda_prepare(eda_handle h, int64_t d, int64_t n, int64_t k,
                       const double* H_W, int64_t ldw, const double* H_B, int64_t ldb,
                       eda_dtype storage);

/* Exponential-vector product of Theorem 3.1:
 *     Out = e^{-s} exp(c S_which) V,   s = max(0, c * lambda_max(S_which)),
 * with s written to *log_scale (host) so that exp(c S) V = e^{s} Out.
 * V: device d x b (ldv >= d); Out: device d x b (ldo >= d), must not overlap V.
 * vdtype: EDA_F64 (V and Out float64), EDA_F32 (float32) or, with bfloat16
 * or FP8 storage, EDA_BF16 (bfloat16; products exact, sums in float32 per
 * 32 rows and float64 beyond, Out rounded once to bfloat16); the factor is
 * read in the storage type of eda_prepare.
 * Stream-ordered; synchronises only when a core for a new c must be built. */
eda_status eda_expmv(eda_handle h, eda_which which, double c, int64_t b,
                     const void* V, int64_t ldv, void* Out, int64_t ldo, eda_dtype vdtype,
                     double* log_scale);

/* Composite operator products (3.16) / (3.2), scaled:
 *     Out = e^{-s} M V  (EDA_FORM_LANCZOS_M)  or  Out = e^{-s} A V  (EDA_FORM_ARNOLDI_A),
 * s = lambda_max(S_B) written to *log_scale (host).  Two streaming passes over
 * P = [H_W H_B].  Same buffer rules as eda_expmv.  Stream-ordered. */
eda_status eda_opmv(eda_handle h, eda_form form, int64_t b,
                    const void* V, int64_t ldv, void* Out, int64_t ldo, eda_dtype vdtype,
                    double* log_scale);

/* eda_opmv without any device allocation, for callers that cannot allocate
 * (work under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, result and stream ordering as eda_opmv, the
 * same launches in the same order (identical bits).  The product's scratch
 * (partial sums, P^T V and the core product) is a static 32 MiB device
 * array per device, shared by every call on that device: calls that overlap
 * on one device race.  EDA_ERR_ARG when a product needs more scratch than
 * that (8 (n + k) b (c + g + 2) bytes, c the row chunks of P^T V, about
 * d / 2048 for long factors, g <= 33 the column groups of the core product:
 * with b = 8 and n + k = 2048 up to d of about 450 000); EDA_ERR_STATE for
 * the Arnoldi form before its core exists (eda_opmv with EDA_FORM_ARNOLDI_A
 * builds it). */
eda_status eda_opmv_noalloc(eda_handle h, eda_form form, int64_t b, const void* V, int64_t ldv,
                            void* Out, int64_t ldo, eda_dtype vdtype, double* log_scale);

/* Algorithm 3: t dominant eigenpairs of eq. (1.7).
 * ritz:     host out [t], lambda_i in decreasing order (+inf if > DBL_MAX).
 * ritz_log: host out [t], log lambda_i.
 * X:        device out, d x t float64 (ldx >= d), orthonormal: QR of the
 *           eigenvectors x_i = exp(-S_W/2) y_i in decreasing-lambda order, each
 *           column's largest-magnitude entry positive.
 * resid:    host out [t], final residual of each Ritz pair of M, measured
 *           explicitly with one more operator product (measure from opts).
 * info:     host out, may be NULL.
 * Requires 1 <= t <= 128, t < d and t + 2b <= max_basis <= d.
 * The Krylov phase (block Lanczos with thick restart on e^{-s} M) runs with
 * the storage type of P and the basis type opts.krylov_dtype, and stops when
 * every pair has estimated residual <= max(tol, 10 u theta_1/theta_i), u the
 * larger unit roundoff of the two types.  A float64 stage follows: explicit
 * residuals with the float64 operator and, while some pair misses
 * max(tol, 10 u64 theta_1/theta_i), refinement passes (Rayleigh-Ritz on the
 * Ritz block and its residual block), at most opts.max_refine of them.
 * EDA_ERR_NOCONV if max_iter or max_refine is exhausted (outputs still
 * written).
 * With opts.form = EDA_FORM_ARNOLDI_A the eigenvectors of A = exp(-S_W)
 * exp(S_B) (eq. 3.1) are computed directly, by block Lanczos in the
 * exp(S_W) inner product (A is self-adjoint in it), keeping exp(S_W) V
 * beside the basis V; each block step is one product with e^{-s} A (core
 * C_A of eq. 3.2) and one with exp(S_W) (the H_W columns of P), about 1.5 to
 * 2 times the traffic of a Lanczos step.  That form runs in float64 only
 * (krylov_dtype EDA_F64; the float64 master of P is used whatever the
 * storage type), has no refinement stage, needs ||H_W^T H_W||_1 <= 12 ln 10
 * and t + 2b <= max_basis <= n - 1 - b (rounded down to a multiple of b; the
 * default is capped there), and resid[i] is the exp(-S_W)-norm of
 * e^{-s} exp(S_B) x_i - theta_i exp(S_W) x_i for exp(S_W)-normalised x_i,
 * relative as in opts.resmode (equal to the Lanczos form's residual of the
 * same pair).  EDA_ERR_NOCONV also when a block loses rank before the
 * tolerance is met.
 * With opts.form = EDA_FORM_JD_M the same pairs of e^{-s} M come from block
 * Jacobi-Davidson (one of the further solvers named in Section 5): every
 * outer step takes the Rayleigh-Ritz pairs of the search space, solves the
 * projected correction equation (I - Y Y^T)(e^{-s} M - theta_i I)(I - Y Y^T)
 * z_i = -r_i for up to b unconverged pairs by 4 GMRES steps (one block
 * product each), and restarts to the t + b leading Ritz vectors plus the
 * corrections.  Float64 only (krylov_dtype EDA_F64; the float64 master of P
 * is used whatever the storage type), max_iter counts outer steps (default
 * 1000), max_basis is unused (the search space holds t + 2b columns, t + 2b
 * <= d), no refinement stage; stopping test, back-transform, outputs and
 * resid as for the Lanczos form.  Synchronises. */
eda_status eda_solve(eda_handle h, int32_t t, double tol, const eda_solve_opts* opt,
                     double* ritz, double* ritz_log, double* X, int64_t ldx,
                     double* resid, eda_info* info);

/* Autotuner of the product passes (Theorem 3.1's two streaming passes over
 * P, and every other tall-skinny product of the same shape class): measures
 * each candidate launch shape for a d x N matrix stored as `storage` and a
 * block of b float64 columns (1 <= b <= 16) on the handle's device, and
 * records the fastest for the shape class (ceil(log2 d), ceil(log2 N),
 * entry size) in a process-wide table used by every later launch; when the
 * environment variable EDA_TUNE_CACHE names a file, the table is read from
 * it once and rewritten after each tuning.  eda_solve_batched tunes the
 * class of its largest problem by itself (EDA_AUTOTUNE=0 disables that).
 * Outputs (host, each may be NULL): *tn_steps = 64-row steps per wave of the
 * P^T V pass (1, 2, 4 or 8); *nn_tile = configuration of the P Z pass (0..3,
 * -1 for FP8/bfloat16 storage, which has one shape); us[0], us[1] = their
 * measured times in microseconds.  Results of the products do not depend on
 * the shapes beyond the order of partial sums.  Synchronises. */
eda_status eda_autotune(eda_handle h, int64_t d, int64_t N, int32_t b, eda_dtype storage,
                        int32_t* tn_steps, int32_t* nn_tile, double* us);

/* Reduced direct solve of eq. (1.7): the same outputs as eda_solve, computed
 * without iteration.  Both exponentials are the identity plus a term in
 * span P (Theorem 3.1), so e^{-s} M restricted to span P is the r x r
 * matrix K = e^{-s} I + F^T C F (r = rank P; F from the eigendecomposition
 * of the Gram matrix P^T P, C the core of the product e^{-s} M): one dense
 * eigensolve of size n + k, one of size r, small GEMMs and three streaming
 * passes.  Uses the float64 factors of the preparation.  resid[i] is
 * ||e^{-s} M y_i - theta_i y_i|| / theta_i (one more product).  Requires
 * 1 <= t <= min(128, rank P), t < d, n + k <= 2048.  info: iters = 0; t_krylov_ms holds the
 * time of the whole solve.  Synchronises. */
eda_status eda_solve_direct(eda_handle h, int32_t t, double* ritz, double* ritz_log, double* X,
                            int64_t ldx, double* resid, eda_info* info);

/* One problem of a batch (eda_solve_batched).  H_W, H_B, X: device;
 * ritz, ritz_log, resid: host arrays of t entries. */
typedef struct {
  int64_t d, n, k;          /* dimension, samples, classes (d >= 2, 2 <= k <= n)   */
  const double* H_W;        /* d x n float64, ldw >= d                            */
  int64_t ldw;
  const double* H_B;        /* d x k float64, ldb >= d                            */
  int64_t ldb;
  int32_t t;                /* wanted pairs, 1 <= t <= 128, t < d                 */
  double tol;               /* residual tolerance as in eda_solve                 */
  double* ritz;             /* host out [t]                                       */
  double* ritz_log;         /* host out [t]                                       */
  double* X;                /* device out, d x t float64, ldx >= d                */
  int64_t ldx;
  double* resid;            /* host out [t]                                       */
} eda_problem;

/* Algorithm 3 for `count` independent problems of different shapes at once
 * (folds and resampled splits of one data set, say).  Every problem is
 * prepared as by eda_prepare (storage type `storage`) and solved as by
 * eda_solve with the options `opt` (start_block must be NULL; problem p
 * draws its start block from seed opt->seed + p), but the kernels of each
 * phase run for all problems in one launch: the problems advance in
 * lockstep, a converged problem drops out of the launches, and the
 * argument arrays of a step are copied to the device in one transfer.
 * infos, statuses: host arrays of `count` entries (may be NULL).  Returns
 * EDA_OK when every problem succeeded, else the first failing status
 * (argument errors are reported before any work is done).  With narrow
 * storage or a float32 basis, a problem whose float64 refinement passes
 * stall continues by eda_solve in float64 on its own handle, with its
 * float64 master as the storage (no new Gram or cores) and a start block
 * mixed from its refined Ritz block (EDA_WARN_FALLBACK; its block steps,
 * restarts, passes, products, bytes and times are added to the problem's
 * info).  Uses the
 * handle's stream and workspaces; does not change the handle's own
 * preparation.  Synchronises. */
eda_status eda_solve_batched(eda_handle h, int32_t count, const eda_problem* probs,
                             eda_dtype storage, const eda_solve_opts* opt, eda_info* infos,
                             eda_status* statuses);

/* Gram matrix G = P^T P of the current preparation (float64, N x N with
 * N = n + k, P = [H_W H_B]); G: device out (ldg >= N).  Stream-ordered. */
eda_status eda_gram(eda_handle h, double* G, int64_t ldg);

/* The stored factor P = [H_W H_B] of the current preparation (factor
 * ingest, eqs. (1.1)-(1.2) in the storage encoding of eda_prepare), for
 * checks of the byte-level encoding: out (device, ld ldo >= d) receives the
 * d x (n + k) entries column-major in the storage type (float64, float32,
 * bfloat16 codes as uint16, E4M3 codes as uint8); for EDA_FP8_E4M3, scales
 * (device, n + k float64, may be NULL) receives the per-column scales, so
 * that P(:, j) ~ scales[j] * decode(out(:, j)).  Stream-ordered. */
eda_status eda_factor_codes(eda_handle h, void* out, int64_t ldo, double* scales);

/* Symmetric eigensolver used for the Gram and Rayleigh-Ritz matrices:
 * A = Z diag(w) Z^T for symmetric A (n x n float64, device, lda >= n, only
 * the lower triangle is read; A is not modified).  w: device out [n]
 * ascending; Z: device out n x n (ldz >= n), orthonormal columns.
 * 1 <= n <= 2048.  Synchronises. */
eda_status eda_syev(eda_handle h, int64_t n, const double* A, int64_t lda,
                    double* w, double* Z, int64_t ldz);

/* Nearest-neighbour classification in the EDA subspace (Section 3.3): the
 * distance between training sample x_i and testing sample y_j is
 * d_ij = ||X^T (x_i - y_j)||_2 for the orthonormal d x t matrix X (as
 * returned by eda_solve), and testing sample j takes the label of the
 * training sample with the smallest d_ij (1-NN; on equal distances the
 * smallest index, a choice the paper leaves open).  X (ldx >= d), train
 * (d x n_train, ldtr >= d), test (d x n_test, ldte >= d): float64, device,
 * column-major; train_labels: device int32 [n_train].  Outputs (device):
 * pred[n_test] = train_labels[nn_index[j]], nn_index[n_test], nn_dist[n_test]
 * = min_i d_ij.  1 <= t <= min(d, 1024), n_train >= 1, 1 <= n_test < 2^31.  Independent
 * of the preparation; uses the handle's stream and workspaces; stream-ordered
 * (no synchronisation).  A testing sample whose distances are all NaN gets
 * index and label -1 and distance NaN. */
eda_status eda_nn_classify(eda_handle h, int64_t d, int64_t t, const double* X, int64_t ldx,
                           int64_t n_train, const double* train, int64_t ldtr,
                           const int32_t* train_labels, int64_t n_test, const double* test,
                           int64_t ldte, int32_t* pred, int64_t* nn_index, double* nn_dist);

#ifdef __cplusplus
}
#endif

#endif /* EDA_H_ */
