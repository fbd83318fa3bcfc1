/*
 * tla.h -- C ABI of libtla, batched small dense solvers for MI355X (gfx950).
 *
 * The three operations are those of the paper's Fig. 2 (caption): for square
 * n x n matrices,
 *   potrf : X^T X = A      A symmetric positive definite, X upper triangular
 *   trsyl : L X + X U = C  L lower triangular, U upper triangular
 *   trlyap: L X + X L^T = S   L lower triangular, S and X symmetric
 * taken literally as printed (plus signs, right-hand side on the right).
 * The paper generates one routine per size n and picks among algorithm
 * variants by autotuning (Generator structure paragraph); here every call
 * handles a batch of independent instances, each with its own n <= n_max.
 *
 * Storage: column-major, element (i,j) of instance b at M[b][i + j*ld[b]].
 * Referenced triangles: potrf reads/writes the upper triangle of A (the
 * strict lower part is never touched); trsyl reads the lower triangle of L
 * and the upper triangle of U, reads C and overwrites it with X; trlyap reads
 * the lower triangles of L and S and overwrites S with the full symmetric X.
 *
 * Ownership: every array argument of a compute call (n, ld*, the pointer
 * arrays, the matrices, info, stat, descriptors) is DEVICE memory owned by the
 * caller and must stay valid until the call's work on the handle's stream has
 * finished.  The handle owns its workspace, graph cache, tuning table and MLP
 * weights.  Compute calls are asynchronous on the handle's stream; info[] and
 * stat[] are valid after the stream has been synchronised.
 *
 * Errors: the return status covers what the host can check (null handle or
 * pointers with batch > 0, batch < 0, n_max < 0 or above the supported
 * maximum, an unknown precision, HIP failures).  Per-instance problems go to
 * info[b]:
 *    0   success
 *   -p   argument p of instance b is invalid (-1: n[b] < 0 or n[b] > n_max,
 *        -2: a leading dimension below max(1, n[b])); the instance is skipped
 *    k>0 potrf: the leading minor of order k is not positive definite (pivot
 *        <= 0 or NaN) in the precision that ran last; A is then unspecified.
 *        trsyl/trlyap: 1 + (i + j*n) of the first zero denominator
 *        l_ii + u_jj (resp. l_ii + l_jj) in column-major order; X unspecified.
 *   -3   (ragged batches only) the descriptor names no known operation
 *   -4   (general equations only) a coefficient has complex eigenvalues
 *   -5   (general equations only) the Schur reduction did not converge, or a
 *        coefficient holds a non-finite entry
 * n[b] = 0 is a quick return with info 0.  Nothing crosses the ABI as an
 * exception.
 */
#ifndef TLA_H
#define TLA_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tla_ctx *tla_handle;

typedef enum {
  TLA_OK = 0,
  TLA_E_ARG = 1,          /* host-checkable argument error */
  TLA_E_HIP = 2,          /* a HIP runtime call failed */
  TLA_E_NOMEM = 3,        /* workspace allocation failed */
  TLA_E_UNSUPPORTED = 4   /* precision / size / option not built */
} tla_status;

/* Arithmetic of a call.  Inputs and outputs are FP64 for every value.  The
 * MIXED_* modes solve in FP32 (tile updates in FP32, FP16 or BF16 on the
 * matrix cores, FP32 accumulate) and refine in FP64: the residual, the
 * correction accumulation and the fallback for refinement that does not
 * converge run in FP64.  The paper itself computes in FP64 only. */
typedef enum { TLA_F64 = 0, TLA_MIXED_F32 = 1, TLA_MIXED_F16 = 2, TLA_MIXED_BF16 = 3 } tla_prec;

typedef enum { TLA_POTRF = 0, TLA_TRSYL = 1, TLA_TRLYAP = 2 } tla_op;

/* stat.flags bits */
#define TLA_STAT_CONVERGED 1   /* refinement reached the tolerance */
#define TLA_STAT_FALLBACK  2   /* refinement stalled or ran out of steps; FP64 solve used */
#define TLA_STAT_BREAKDOWN 4   /* low-precision solve broke down; FP64 solve used */
#define TLA_STAT_NONFINITE 8   /* a non-finite input value was seen */

/* Per-instance refinement record (device memory, optional).  eta is the final
 * FP64 backward error (see tla_set_refine); iters the number of corrections. */
typedef struct { int iters; int flags; double eta; } tla_stat;

/* Ragged work item: one instance of any operation (device memory array).
 *   potrf : a = A,             lda
 *   trsyl : a = L, b = U, c = C/X, lda = ldl, ldb = ldu, ldc
 *   trlyap: a = L, c = S/X,    lda = ldl, ldc = lds        */
typedef struct {
  int op, n;
  int lda, ldb, ldc, pad_;
  double *a, *b, *c;
} tla_desc;

/* ---------------------------------------------------------------- handles */
/* Create a handle bound to HIP device `device` (made current).  The handle's
 * stream starts as the device's null stream. */
tla_status tla_create(tla_handle *h, int device);
tla_status tla_destroy(tla_handle h);
/* Subsequent work is enqueued on `stream` (a hipStream_t passed as void*). */
tla_status tla_set_stream(tla_handle h, void *stream);
/* Synchronise the handle's stream. */
tla_status tla_sync(tla_handle h);

/* --------------------------------------------------------- batched solves */
/* Upper Cholesky X^T X = A (paper Fig. 2a): overwrites the upper triangle of
 * each A[b] with X.  n, lda, info: int[batch]; A: double*[batch]; stat:
 * tla_stat[batch] or NULL. */
tla_status tla_potrf_batched(tla_handle h, tla_prec prec, int batch, int n_max,
                             const int *n, double *const *A, const int *lda,
                             int *info, tla_stat *stat);

/* Triangular Sylvester L X + X U = C (paper Fig. 2c): overwrites each C[b]
 * with X. */
tla_status tla_trsyl_batched(tla_handle h, tla_prec prec, int batch, int n_max,
                             const int *n, const double *const *L, const int *ldl,
                             const double *const *U, const int *ldu,
                             double *const *C, const int *ldc, int *info, tla_stat *stat);

/* Triangular Lyapunov L X + X L^T = S (paper Fig. 2b): reads the lower
 * triangle of each S[b] and overwrites the full S[b] with the symmetric X. */
tla_status tla_trlyap_batched(tla_handle h, tla_prec prec, int batch, int n_max,
                              const int *n, const double *const *L, const int *ldl,
                              double *const *S, const int *lds, int *info, tla_stat *stat);

/* Solve with the upper Cholesky factor, FP64: for every instance b,
 * B_b := (X_b^T X_b)^{-1} B_b by forward substitution with X_b^T and back
 * substitution with X_b.  This is the consumer of the factorization
 * (Fig. 2a) that the paper's motivation lists next to it among the LAPACK
 * building blocks.
 *   X[b]: the n[b] x n[b] upper factor as returned by tla_potrf_batched,
 *         column-major with leading dimension ldx[b]; only its upper
 *         triangle is read.
 *   B[b]: n[b] x nrhs[b] right-hand sides, column-major with leading
 *         dimension ldb[b]; overwritten with the solution.
 *   0 <= n[b] <= n_max, 0 <= nrhs[b] <= nrhs_max.  All arrays (pointer
 *   arrays included) are device memory owned by the caller.
 * info[b]: 0; -1 bad n or nrhs; -2 ldx or ldb < max(1, n); k > 0 when the
 * factor's diagonal entry x_kk (1-based) is zero, B_b then left unchanged.
 * Asynchronous on the handle's stream. */
tla_status tla_potrs_batched(tla_handle h, int batch, int n_max, const int *n, int nrhs_max, const int *nrhs,
                             const double *const *X, const int *ldx, double *const *B, const int *ldb,
                             int *info);

/* Inverse from the upper Cholesky factor, FP64: Y_b := (X_b^T X_b)^{-1}, the
 * full n[b] x n[b] matrix (symmetric up to rounding), written to the
 * caller's Y[b] (column-major, leading dimension ldy[b]) by solving with the
 * factor for the columns of the identity.  X as for tla_potrs_batched.
 * info[b]: 0; -1 bad n; -2 ldx or ldy < max(1, n); k > 0 when x_kk (1-based)
 * is zero, Y_b then the identity.  Asynchronous on the handle's stream. */
tla_status tla_potri_batched(tla_handle h, int batch, int n_max, const int *n, const double *const *X,
                             const int *ldx, double *const *Y, const int *ldy, int *info);

/* FP32-I/O twins of the three batched solves (paper Fig. 2a, 2c, 2b): the
 * same operations, argument roles, layouts, referenced triangles, in-place
 * semantics and info codes as tla_potrf_batched, tla_trsyl_batched and
 * tla_trlyap_batched, on single-precision matrices (float*), computed in
 * single precision (FP32 vector arithmetic for the diagonal tiles, FP32
 * matrix cores for the tile updates).  No refinement and no stat record:
 * the result carries FP32 rounding errors (backward error of order n times
 * the FP32 unit roundoff).  0 <= n[b] <= n_max <= 4096.  All arrays
 * (pointer arrays included) are device memory owned by the caller.
 * Asynchronous on the handle's stream. */
tla_status tla_spotrf_batched(tla_handle h, int batch, int n_max, const int *n, float *const *A, const int *lda,
                              int *info);
tla_status tla_strsyl_batched(tla_handle h, int batch, int n_max, const int *n, const float *const *L,
                              const int *ldl, const float *const *U, const int *ldu, float *const *C,
                              const int *ldc, int *info);
tla_status tla_strlyap_batched(tla_handle h, int batch, int n_max, const int *n, const float *const *L,
                               const int *ldl, float *const *S, const int *lds, int *info);

/* General (non-triangular) Sylvester A X + X B = C and Lyapunov
 * A X + X A^T = S, the equations whose triangular cores are those of the
 * paper's Fig. 2 (the Motivation paragraph names solvers for Sylvester-like
 * equations as the purpose of the triangular kernels).  Bartels-Stewart: the
 * real Schur forms A^T = Z T_A Z^T and B = W T_B W^T are computed on the GPU
 * (Householder Hessenberg reduction, implicit single-shift QR), the
 * right-hand side is transformed to Z^T C W (Z^T S Z), the triangular
 * equation with L = T_A^T and U = T_B (tla_trsyl_batched /
 * tla_trlyap_batched, in the precision `prec`, refined to FP64 as there) is
 * solved in place, and X = Z Y W^T (Z Y Z^T) is written back.
 *   A[b], B[b]: general n[b] x n[b] coefficients, column-major with leading
 *   dimensions lda[b], ldb[b]; read in full, never written.
 *   C[b] (S[b]): right-hand side, column-major with leading dimension ldc[b]
 *   (lds[b]); overwritten with X.  gelyap reads the lower triangle of S and
 *   writes the full, exactly symmetric X.
 *   0 <= n[b] <= n_max <= 64 (n_max above 64: TLA_E_UNSUPPORTED).  All arrays
 *   (pointer arrays included) are device memory owned by the caller.  The
 *   handle keeps the Schur factors in a workspace of its own (4 n_max^2
 *   doubles per instance for gesyl, 2 for gelyap).
 *   Each coefficient is scaled by a power of two before its reduction (its
 *   largest entry into [1/2, 1), exact), so entries of any finite magnitude
 *   are handled, and scaling A, B and C (A and S) by a common power of two
 *   leaves X unchanged bit for bit.
 * The coefficients must have real eigenvalues (the triangular cores are
 * real): info[b] = -4 reports a complex conjugate pair, -5 a QR iteration
 * that did not converge or a non-finite coefficient entry; the instance's
 * right-hand side is then left unchanged.  info[b] = k > 0 reports the first
 * zero denominator lambda_i(A) + lambda_j(B) of the triangular equation
 * (Schur ordering, as for tla_trsyl_batched); X is then unspecified.
 * -1 / -2 as for every call (ld of A, B or C).  stat as for the triangular
 * call (records of the triangular solve).  Asynchronous on the handle's
 * stream. */
tla_status tla_gesyl_batched(tla_handle h, tla_prec prec, int batch, int n_max, const int *n,
                             const double *const *A, const int *lda, const double *const *B,
                             const int *ldb, double *const *C, const int *ldc, int *info,
                             tla_stat *stat);
tla_status tla_gelyap_batched(tla_handle h, tla_prec prec, int batch, int n_max, const int *n,
                              const double *const *A, const int *lda, double *const *S,
                              const int *lds, int *info, tla_stat *stat);

/* Mixed batch of all three operations and uneven n in one persistent launch
 * (captured as a HIP graph and replayed when the same descriptor array, batch
 * and precision come again).  d: tla_desc[batch]. */
tla_status tla_ragged_batched(tla_handle h, tla_prec prec, int batch, int n_max,
                              const tla_desc *d, int *info, tla_stat *stat);

/* Allocation-free variant of tla_ragged_batched, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, work and results as
 * tla_ragged_batched with prec = TLA_F64 (the same class workers and
 * per-instance bodies), but the work-list buffers (cost ranks, key histogram,
 * class counters, queue) live in a fixed 4 MiB device array that each GPU
 * holds until the process ends, set up by tla_create; the call allocates
 * nothing, captures no graph and enqueues its kernels directly on the
 * handle's stream.  Limits: batch <= 1048576 (larger batches return
 * TLA_E_ARG before any work is enqueued), n_max <= 128, prec = TLA_F64 only
 * (the mixed precisions need the handle's workspace: TLA_E_UNSUPPORTED);
 * stat may be NULL.  Every call on one GPU shares that GPU's array, so calls
 * that overlap in time on one GPU (several streams or host threads) race;
 * calls ordered on one stream do not. */
tla_status tla_ragged_batched_noalloc(tla_handle h, tla_prec prec, int batch, int n_max,
                                      const tla_desc *d, int *info, tla_stat *stat);

/* Exact-size kernels (the paper's routines are generated for each input size,
 * Preliminary performance results paragraph).  FP64 calls whose plan solves
 * in place (placement 3, n_max <= 128) can run the same kernel compiled at
 * run time (hiprtc) for n = n_max as a compile-time constant, cached on the
 * handle per (op, n, variant, waves); compiling takes about a third of a
 * second.  Instances with n[b] != n_max take the generic code compiled into
 * the same kernel.  mode 0: off (default); 1: always; 2: where measured
 * faster -- the first call of a key times the plan both ways on synthetic
 * inputs (synchronous, allocates) and keeps the faster for that key.  The
 * kernel source is the library's headers in the csrc directory next to the
 * built library (or in the directory named by TLA_KERNEL_DIR); when they are
 * missing or do not compile, the call uses the ahead-of-time kernel. */
tla_status tla_set_exact_size(tla_handle h, int mode);
/* Exact-size kernels compiled so far on the handle, and compilations that failed. */
tla_status tla_exact_size_stats(tla_handle h, int *compiled, int *failed);

/* ------------------------------------------------------- plans and tuning */
/* A plan names the kernel that solves one (op, n bucket, precision):
 * variant = blocked-algorithm variant (op specific, see tla_variant_name),
 * tile    = diagonal-block size (8 or 16),
 * engine  = 0 vector ALU tile updates, 1 matrix-core (MFMA) tile updates,
 * waves   = wavefronts per instance (1, 2 or 4),
 * place   = 0 stage the triangular coefficients in LDS when they fit,
 *           1 read them through the caches (smaller LDS footprint, more
 *           instances per compute unit; Sylvester and Lyapunov only),
 *           2 (mixed precisions only) also keep the FP64 solution (and,
 *           for the Cholesky factorisation, the FP32 copy of the factor) in
 *           the handle's workspace; its FP64 fallback is then a second launch,
 *           3 (FP64 only; tile 16 with the matrix cores) solve in place in
 *           the caller's matrices in global memory, only the tile solvers'
 *           scratch in LDS (the most instances per compute unit).
 * The launch falls back to a larger place value when LDS does not fit. */
typedef struct { int variant, tile, engine, waves, place; } tla_plan;

/* Which picker chooses plans: the measured tuning table, the MLP cost model
 * (the table remains the fallback), or the built-in default. */
typedef enum { TLA_PICK_DEFAULT = 0, TLA_PICK_TABLE = 1, TLA_PICK_MLP = 2 } tla_picker;

/* Force a plan for (op, prec) on every later call (variant < 0 clears it). */
tla_status tla_set_plan(tla_handle h, tla_op op, tla_prec prec, const tla_plan *plan);
/* Plan the handle would use for (op, n, prec, batch). */
tla_status tla_get_plan(tla_handle h, tla_op op, int n, tla_prec prec, int batch, tla_plan *plan);
/* Number of candidate plans for op and the i-th one (host memory). */
int tla_num_candidates(tla_op op);
tla_status tla_candidate(tla_op op, int i, tla_plan *plan);
const char *tla_variant_name(tla_op op, int variant);

/* Time every candidate plan for each (op, n, prec) of the given lists on
 * synthetic device inputs (batch instances each, `reps` timed launches per
 * candidate) and record the fastest in the handle's tuning table; also
 * stores every measurement.  Synchronous.  ops/ns/precs: host arrays. */
tla_status tla_tune(tla_handle h, int n_ops, const int *ops, int n_ns, const int *ns,
                    int n_precs, const int *precs, int batch, int reps);
/* Measured time (seconds per launch) of one plan, synchronous. */
tla_status tla_time_plan(tla_handle h, tla_op op, int n, tla_prec prec, int batch,
                         const tla_plan *plan, int reps, double *seconds);
/* Tuning table persistence (text, one measurement per line). */
tla_status tla_save_table(tla_handle h, const char *path);
tla_status tla_load_table(tla_handle h, const char *path);
tla_status tla_set_picker(tla_handle h, tla_picker mode);

/* ------------------------------------------------- learned cost model */
/* A small MLP (features -> 64 ReLU -> 64 ReLU -> 1, FP32) predicts the log
 * run time of a plan so that plans can be picked without timing every
 * candidate -- the model-based replacement of autotuning that the paper lists
 * as future work (Limitations and future work paragraph).  It is trained on
 * the GPU, by the library's own forward/backward/Adam kernels, on the
 * measurements in the handle's tuning table; the table remains the fallback,
 * also at sizes outside those the network was trained on (per operation and
 * precision; a network set or loaded from a file covers every size).
 * Parameters are one flat FP32 array (W1[64][F], b1[64], W2[64][64], b2[64],
 * w3[64], b3), F = tla_mlp_num_features().  Host arrays; calls synchronise. */
int tla_mlp_num_params(void);
int tla_mlp_num_features(void);
/* Feature vector of (op, n, prec, batch, plan) into out[F]. */
tla_status tla_mlp_features(tla_op op, int n, tla_prec prec, int batch, const tla_plan *plan, float *out);
tla_status tla_mlp_set_params(tla_handle h, const float *params);
tla_status tla_mlp_get_params(tla_handle h, float *params);
/* Mean squared error of the network on N samples X[N][F] with targets T[N],
 * and its gradient (grad[num_params], may be NULL) and outputs (Y[N], may be
 * NULL), computed by the device kernels. */
tla_status tla_mlp_forward_backward(tla_handle h, int N, const float *X, const float *T, float *loss,
                                    float *grad, float *Y);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the given gradient. */
tla_status tla_mlp_adam_step(tla_handle h, const float *grad, float lr);
/* Train from a seeded initialisation on the tuning table's measurements,
 * leaving out n with n % exclude_mod == 0 when exclude_mod > 0 (held-out
 * sizes); `epochs` full-batch Adam steps; final training loss out. */
tla_status tla_mlp_train(tla_handle h, int epochs, float lr, unsigned long long seed, int exclude_mod,
                         float *final_loss);
/* Predicted seconds per launch of a plan. */
tla_status tla_mlp_predict(tla_handle h, tla_op op, int n, tla_prec prec, int batch, const tla_plan *plan,
                           double *seconds);
tla_status tla_mlp_save(tla_handle h, const char *path);
tla_status tla_mlp_load(tla_handle h, const char *path);
/* The measured autotuner as the fallback and judge of the learned picker:
 * when the network's predicted times of its best candidates lie within a
 * factor (1 + margin) of the best prediction, the picker times those
 * candidates (at most max_timed, best predicted first, on synthetic inputs of
 * the query's op, n, precision and batch, with the autotuner's timer) instead
 * of trusting the network, adds the measurements to the tuning records, keeps
 * the measured winner for that (op, n, precision) and counts a misprediction
 * when the winner is not the network's first choice.  The first pick of such
 * a key is then synchronous.  margin 0 or max_timed < 2 turns the judge off;
 * the default is margin 0.10, max_timed 4.  Setting it (or retraining or
 * loading the network) forgets the kept winners.  Host call. */
tla_status tla_set_picker_judge(tla_handle h, double margin, int max_timed);
/* Picks the judge has timed since the handle was created, and how many of
 * them the network had mispredicted.  Host memory. */
tla_status tla_picker_judge_stats(tla_handle h, int *judged, int *mispredicted);

/* ---------------------------------------------------------- refinement */
/* Refinement tolerance on the backward error eta (default 1e-13) and the
 * maximum number of corrections (default 8). */
tla_status tla_set_refine(tla_handle h, double tau, int max_iter);

const char *tla_status_string(tla_status s);

#ifdef __cplusplus
}
#endif
#endif /* TLA_H */
