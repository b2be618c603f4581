/*
 * nmf.h -- C ABI of the enforced-sparsity NMF library for AMD MI355X (gfx950).
 *
 * The library factors a sparse non-negative term/document matrix A (n x m)
 * as A ~ U V^T with U (n x k) >= 0 and V (m x k) >= 0, minimising
 * ||A - U V^T|| (Eqs. (1)-(2) of Gavin, Gadepally and Kepner, "Enforced Sparse
 * Non-Negative Matrix Factorization").  One iteration is Algorithm 2:
 *   V = A^T U (U^T U)^-1, negatives set to zero, keep the t_v largest;
 *   U = A V (V^T V)^-1,  negatives set to zero, keep the t_u largest;
 * with the "keep the t largest" rule of Section 2 applied to every column of
 * U and V separately (the column-wise variant of Section 4) by default.
 *
 * Conventions shared by every entry point:
 *  - Status codes only; nothing is thrown across the ABI.  nmf_last_error()
 *    returns a message for the last failing call on a handle.
 *  - Dense matrices are row-major, element type given by nmf_config.dtype
 *    (float for NMF_F32, double for NMF_F64).
 *  - "Host or device" pointers: the library asks the HIP runtime which one a
 *    pointer is and copies accordingly.  The caller keeps ownership of every
 *    array it passes; nothing is retained after a call returns.
 *  - All device memory the library uses lives in one caller-provided
 *    workspace (sized by nmf_workspace_size); the library never allocates
 *    device memory itself.
 *  - Asynchronous calls enqueue work on the handle's HIP stream and return at
 *    once.  Calls marked "synchronizes" wait for that stream.
 *  - Numerical failures detected on the device (NMF_ERR_NOT_SPD,
 *    NMF_ERR_NONFINITE) are sticky: they surface at the next synchronizing
 *    call, and every later kernel of the handle does nothing.
 *  - A handle is not thread-safe; use one handle per thread.
 */
#ifndef NMF_H
#define NMF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmf_handle nmf_handle;

typedef enum {
  NMF_OK = 0,
  NMF_ERR_INVALID_ARG = -1,   /* bad size, null pointer, malformed CSR      */
  NMF_ERR_INVALID_INPUT = -2, /* negative, NaN or Inf value in A or factors  */
  NMF_ERR_UNSUPPORTED = -3,   /* k > 128, n or m >= 2^29, a dense factor of
                                 4 GiB or more (rows x k padded to 64 bytes),
                                 unknown dtype or mode                        */
  NMF_ERR_NOT_SPD = -4,       /* Gram matrix not positive definite           */
  NMF_ERR_NONFINITE = -5,     /* NaN/Inf produced (e.g. ||U_i|| = 0 in R)    */
  NMF_ERR_DEVICE = -6,        /* a HIP runtime call failed                   */
  NMF_ERR_STATE = -7,         /* call not valid in the handle's state        */
  NMF_ERR_WORKSPACE = -8      /* workspace too small or misaligned           */
} nmf_status;

/* Sparsity enforcement mode. */
enum {
  NMF_MODE_COLUMN = 0, /* t largest per column (Section 4)                    */
  NMF_MODE_NONE = 1,   /* projection only: Algorithm 1                        */
  NMF_MODE_WHOLE = 2   /* t largest of the whole matrix (Algorithm 2 printed);
                          ties at the t-th value go to the lowest (row, column)
                          in row-major order                                  */
};

/* Arithmetic type of A, U, V and of the sparse products.  The k x k Gram
 * factorisation and the solve are always float64. */
enum { NMF_F32 = 0, NMF_F64 = 1 };

/* nmf_config.flags */
enum {
  NMF_FLAG_NO_METRICS = 1, /* skip the per-iteration E and R (history keeps nnz) */
  NMF_FLAG_NO_HOT = 2      /* keep every term in the V-half sparse stream (float32:
                              by default the densest terms' nonzeros are stored as
                              a dense block multiplied on the matrix cores; the
                              results agree to float32 rounding) */
};

typedef struct {
  int64_t n;     /* terms (rows of A, rows of U), 1 <= n < 2^29   */
  int64_t m;     /* documents (columns of A, rows of V), < 2^29   */
  int32_t k;     /* topics, 1 <= k <= min(n, m, 128)               */
  int32_t mode;  /* NMF_MODE_*                                     */
  int64_t t_u;   /* kept entries per column of U (>= 1)            */
  int64_t t_v;   /* kept entries per column of V (>= 1)            */
  int32_t dtype; /* NMF_F32 | NMF_F64                              */
  int32_t flags; /* NMF_FLAG_*                                     */
} nmf_config;

/* Bytes of device workspace a handle for this configuration and this many
 * nonzeros of A needs.  Pure host computation; no device is touched.
 * Errors: NMF_ERR_INVALID_ARG / NMF_ERR_UNSUPPORTED for a bad config. */
nmf_status nmf_workspace_size(const nmf_config* cfg, int64_t nnz, size_t* bytes);

/* Create a handle for A given in CSR over term rows: a_rowptr[n+1] (int64,
 * a_rowptr[0] = 0, non-decreasing, a_rowptr[n] = nnz), a_col[nnz] (int32,
 * strictly increasing within a row, in [0, m)), a_val[nnz] (dtype, finite,
 * >= 0).  u0 is the initial guess U0 (n x k, finite, >= 0) of Algorithms 1-2;
 * v0 (m x k) is optional (NULL) and only serves nmf_error before the first
 * step.  workspace/ws_bytes: device memory of at least nmf_workspace_size()
 * bytes, 256-byte aligned, owned by the caller and not touched by anyone else
 * while the handle lives.  hip_stream: the hipStream_t every kernel of this
 * handle runs on (NULL = the default stream).  Copies A, U0 (and V0) into the
 * workspace, builds the transposed copy of A, and synchronizes.
 * Errors: INVALID_ARG (malformed CSR, sizes), INVALID_INPUT (negative or
 * non-finite values, ||A|| = 0), UNSUPPORTED, WORKSPACE, DEVICE.  On error
 * *out is NULL. */
nmf_status nmf_create(const nmf_config* cfg, const int64_t* a_rowptr, const int32_t* a_col,
                      const void* a_val, int64_t nnz, const void* u0, const void* v0,
                      void* workspace, size_t ws_bytes, void* hip_stream, nmf_handle** out);

/* Size of the static workspace behind nmf_create_static, per device. */
#define NMF_STATIC_WORKSPACE_BYTES (64ull << 20)

/* nmf_create for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same
 * handle, with the library's static device workspace of
 * NMF_STATIC_WORKSPACE_BYTES (64 MiB; one array per device, held until the
 * process ends) in place of a caller's workspace.  Arguments, layouts,
 * ownership of the inputs and behaviour are those of nmf_create.  Allocates
 * no device memory: no hipMalloc/hipFree/hipHostMalloc and no allocating
 * library call (host-side set-up uses the C++ heap as nmf_create does).  The
 * workspace keeps whatever the previous handle left; creation clears what
 * must start at zero.  One live handle per device owns it: a second call on
 * the same device before nmf_destroy of the first returns NMF_ERR_STATE
 * (calls on the one handle from several threads race, as for any handle).
 * Errors: those of nmf_create, plus WORKSPACE when nmf_workspace_size()
 * exceeds NMF_STATIC_WORKSPACE_BYTES and STATE as above. */
nmf_status nmf_create_static(const nmf_config* cfg, const int64_t* a_rowptr, const int32_t* a_col,
                             const void* a_val, int64_t nnz, const void* u0, const void* v0, void* hip_stream,
                             nmf_handle** out);

/* Enqueue `iters` iterations of Algorithm 2 (V half-step first, from the
 * current U), each followed by R and E of Section 3.1 unless
 * NMF_FLAG_NO_METRICS.  Asynchronous.  iters >= 0. */
nmf_status nmf_als_step(nmf_handle* h, int32_t iters);

/* One half-step only: which = 0 solves V from the current U (Algorithm 2
 * steps 1-2), which = 1 solves U from the current V (steps 3-4; the previous
 * U becomes U_{i-1}).  No metrics are recorded.  Asynchronous. */
nmf_status nmf_half_step(nmf_handle* h, int32_t which);

/* Relative error E = ||A - U V^T||_F / ||A||_F (Section 3.1) of the current
 * U and V.  Synchronizes.  NMF_ERR_STATE if no V exists yet (no step taken
 * and no v0 given). */
nmf_status nmf_error(nmf_handle* h, double* E);

/* Relative residual R = ||U_i - U_{i-1}||_F / ||U_i||_F (Section 3.1) of the
 * last completed iteration.  Synchronizes.  NMF_ERR_STATE before the first
 * iteration. */
nmf_status nmf_residual(nmf_handle* h, double* R);

/* Per-iteration record, oldest first, of up to `cap` of the most recent
 * iterations: E, R, nnz(U), nnz(V) (any of the arrays may be NULL).  *len
 * receives the number written.  Synchronizes.  With NMF_FLAG_NO_METRICS, E
 * and R are NaN. */
nmf_status nmf_history(nmf_handle* h, double* E, double* R, int64_t* nnz_u, int64_t* nnz_v,
                       int32_t cap, int32_t* len);

/* Fields of the per-iteration record (nmf_history_field). */
enum {
  NMF_HIST_E = 0,        /* relative error E (Section 3.1)                          */
  NMF_HIST_R = 1,        /* relative residual R (Section 3.1)                       */
  NMF_HIST_NNZ_U = 2,    /* entries stored in U after the iteration                 */
  NMF_HIST_NNZ_V = 3,    /* entries stored in V                                     */
  NMF_HIST_DEAD_U = 4,   /* dead topics (all-zero columns) of U                     */
  NMF_HIST_DEAD_V = 5,   /* dead topics of V                                        */
  NMF_HIST_COND_U = 6,   /* conditioning of U^T U at the end of the iteration: the
                            largest G_cc (G^-1)_cc over live topics (1 for
                            orthogonal columns; a lower bound of the condition
                            number; NaN after nmf_sequential, which forms only
                            block inverses)                                         */
  NMF_HIST_COND_V = 7,   /* the same for V^T V (the matrix the U half solved with)  */
  NMF_HIST_GATHERED_V = 8, /* factor entries the V-half product gathered since the
                            previous record: the sum over the streamed nonzeros of A
                            of the stored entries of the U row each hits (the hot
                            block's product is dense and not counted)               */
  NMF_HIST_GATHERED_U = 9, /* the same for the U-half product (rows of V)           */
  NMF_HIST_NUM_FIELDS = 10
};

/* One field (NMF_HIST_*) of the per-iteration record, oldest first, for up to
 * `cap` of the most recent iterations into out (host); *len receives the
 * number written.  Synchronizes.  Errors: INVALID_ARG (unknown field, NULL
 * out or len, cap < 0). */
nmf_status nmf_history_field(nmf_handle* h, int32_t field, double* out, int32_t cap, int32_t* len);

/* Largest nnz(U) + nnz(V) held at the end of any half-step so far, counting
 * U0 (the storage high-water mark of Section 3.2).  Synchronizes. */
nmf_status nmf_max_nnz(nmf_handle* h, int64_t* max_nnz_uv);

/* Copy the current factors out as dense row-major arrays (host or device):
 * u_dense n x k, v_dense m x k; either may be NULL.  Synchronizes. */
nmf_status nmf_get_factors(nmf_handle* h, void* u_dense, void* v_dense);

/* Export the current factors in the row-compressed sparse form the library
 * stores: row_ptr int32[rows+1], topic uint8[nnz], val dtype[nnz], topics
 * ascending within a row.  Pass NULL arrays to query only *nnz.  Host or
 * device pointers.  which = 0 for U, 1 for V.  Synchronizes. */
nmf_status nmf_get_sparse(nmf_handle* h, int32_t which, int32_t* row_ptr, uint8_t* topic,
                          void* val, int64_t* nnz);

/* Replace the state: u (n x k, required), u_prev (n x k, U_{i-1} for the
 * next residual; NULL = same as u), v (m x k, NULL = keep).  Dense row-major,
 * host or device, finite and >= 0; zeros are not stored.  Used to resume a
 * run or to start a half-step from a given state.  Synchronizes.
 * Errors: INVALID_ARG, INVALID_INPUT. */
nmf_status nmf_set_factors(nmf_handle* h, const void* u, const void* u_prev, const void* v);

/* The clamped pre-selection matrix of the last half-step of each kind:
 * which = 0: max(0, A^T U (U^T U)^-1) (m x k); which = 1: max(0, A V (V^T V)^-1)
 * (n x k).  Dense row-major, host or device.  Synchronizes. */
nmf_status nmf_get_pre(nmf_handle* h, int32_t which, void* dst);

/* Squared loss L = ||A - U V^T||_F^2 = ||A||^2 - 2 tr(U^T A V) + tr(U^T U V^T V)
 * (the squared objective of Eq. (2)) for caller-given dense U (n x k) and
 * V (m x k), device pointers of the handle's dtype.  *loss_dev is a device
 * float64.  Uses the handle's copy of A.  Synchronizes with the handle's
 * stream before (to read the sticky status: while a numerical error is
 * pending the products would be skipped) and after (a non-finite product
 * is reported here).  Errors: INVALID_ARG (NULL or host pointer), the
 * pending sticky status, NONFINITE, DEVICE. */
nmf_status nmf_loss_fwd(nmf_handle* h, const void* U, const void* V, double* loss_dev);

/* Gradient of that loss scaled by the device scalar *g_scale (float64; pass
 * NULL for 1): gU = g (-2 A V + 2 U V^T V), gV = g (-2 A^T U + 2 V U^T U).
 * Device pointers, dtype of the handle, gU n x k and gV m x k (either may be
 * NULL to skip).  Synchronizes before and after, as nmf_loss_fwd.
 * Errors: as nmf_loss_fwd. */
nmf_status nmf_loss_bwd(nmf_handle* h, const void* U, const void* V, const double* g_scale,
                        void* gU, void* gV);

/* Stages of one iteration, for nmf_profile_read. */
enum {
  NMF_STAGE_SPMM_V = 0,   /* A^T U, solve, clamp (Algorithm 2 step 1)      */
  NMF_STAGE_SELECT_V = 1, /* per-column top-t_v (step 2)                   */
  NMF_STAGE_REPACK_V = 2, /* sparse repack of V                            */
  NMF_STAGE_GRAM_V = 3,   /* V^T V, Cholesky, inverse                      */
  NMF_STAGE_SPMM_U = 4,   /* A V, solve, clamp (step 3)                    */
  NMF_STAGE_SELECT_U = 5, /* per-column top-t_u (step 4)                   */
  NMF_STAGE_REPACK_U = 6,
  NMF_STAGE_GRAM_U = 7,
  NMF_STAGE_METRICS = 8,  /* R and E of Section 3.1                        */
  NMF_NUM_STAGES = 9
};

/* Measurement aid, not part of the method: while enabled (enable != 0),
 * every stage that nmf_als_step enqueues is bracketed by HIP events on the
 * handle's stream.  Enabling clears the totals.  Host-side events only; no
 * device memory is allocated. */
nmf_status nmf_profile(nmf_handle* h, int32_t enable);

/* As nmf_profile, for the stages whose bit is set in `stages` (bit s =
 * NMF_STAGE_s; 0 disables).  An event is recorded only where a bracketed
 * stage begins or ends, so the other stages run back to back, as without
 * profiling (each recorded event delays the next launch by a few
 * microseconds).  NMF_ERR_INVALID_ARG for bits at or above NMF_NUM_STAGES. */
nmf_status nmf_profile_stages(nmf_handle* h, uint32_t stages);

/* Summed event time (milliseconds) and number of launches per stage since
 * profiling was enabled; arrays of n_stages entries (<= NMF_NUM_STAGES).
 * Synchronizes. */
nmf_status nmf_profile_read(nmf_handle* h, double* ms, int64_t* count, int32_t n_stages);

/* Tuning parameters (performance only; results stay within the documented
 * tolerance and are reproducible for a given setting). */
enum {
  NMF_PARAM_SPARSE_ROW_V = 0, /* V half through the SpMM stream (float64, or
                                 k > 64): U rows with <= this many entries
                                 are gathered entry by entry, denser rows
                                 whole (0..128; default 1).  The fused
                                 V-half kernel (float32, k <= 64) reads
                                 every nonempty row whole and ignores it    */
  NMF_PARAM_SPARSE_ROW_U = 1, /* U half: the same for rows of V (default 1;
                                 3 when k > 64)                             */
  NMF_PARAM_WIDE_V = 2,       /* V half SpMM step form: 0 = 64 nonzeros per
                                 step with loads only on the lanes that need
                                 them (default; suits factors whose gathered
                                 rows are mostly dense), 1 = 128 nonzeros per
                                 step with every load issued on all lanes
                                 (suits very sparse gathered rows; default
                                 when k > 64); not used by the fused V-half
                                 kernel                                     */
  NMF_PARAM_WIDE_U = 3,       /* U half: the same (default 1)               */
  NMF_PARAM_WAVES_V = 4,      /* V half: waves per block, 1/2/4/8/16 (default
                                 16; fewer when the k x k inverse and the
                                 wave buffers exceed the LDS)               */
  NMF_PARAM_WAVES_U = 5,      /* U half: the same (default 8; 16 when
                                 k > 64)                                    */
  NMF_NUM_PARAMS = 6
};

/* Set a tuning parameter of a handle (applies to later launches).  A problem
 * of a batch takes new values through nmf_batch_set_param.  The parameters
 * change which kernels and launch shapes run; results change at most by
 * float32 summation order (the waves setting not at all).
 * Errors: INVALID_ARG for an unknown parameter or a value out of range. */
nmf_status nmf_set_param(nmf_handle* h, int32_t param, int64_t value);

/* Sequential ALS (Algorithm 3, Section 4): find the k topics k2 at a time.
 * Block b (b = 0 .. k/k2 - 1) solves columns [b k2, (b + 1) k2) of U and V
 * for `iters` iterations while the earlier columns stay fixed, with the
 * deflated least-squares solves of Eqs. (seq-V)/(seq-U):
 *   V2 = (A^T U2 - V1 (U1^T U2)) (U2^T U2)^-1,  U2 = (A V2 - U1 (V1^T V2)) (V2^T V2)^-1,
 * each clamped at zero and cut to the t_v / t_u largest entries of every
 * column (the handle's per-column rule; NMF_MODE_NONE: no cut).  Every block
 * starts from the same initial guess: the first k2 columns of U when the
 * call begins (for a fresh handle, of U0; the other columns of U0 are not
 * used).  Block 0 is Algorithm 2 on those k2 topics.  U and V keep all k
 * columns (later blocks' columns are zero until solved); each iteration
 * records E and R (Section 3.1) of the full factors in the history, R
 * against U as it stood when the iteration began.  k2 must divide k.  With
 * k2 < k the block's sparse products gather and store only its k2 columns of
 * the fixed factor (the U half skips the nonzeros whose row of V stores
 * nothing in them).  Asynchronous.  Errors: INVALID_ARG, UNSUPPORTED (NMF_MODE_WHOLE),
 * NOT_SPD (a block's Gram matrix; sticky, reported at the next sync). */
nmf_status nmf_sequential(nmf_handle* h, int32_t k2, int32_t iters);

/* Apply the top-t rule once to the current U (t_u) and V (t_v): mode
 * NMF_MODE_COLUMN per column (Section 4), NMF_MODE_WHOLE over the whole
 * factor (Section 2), with the tie-breaks of the iteration; their Gram
 * matrices are rebuilt.  With a handle in NMF_MODE_NONE this is the
 * "enforce sparsity after ALS" of Section 3.2 (Algorithm 1 to the end, then
 * one top-t).  Later iterations continue from the sparsified factors under
 * the handle's own mode.  The next nmf_error computes E of the new factors.
 * Synchronizes.  Errors: INVALID_ARG, STATE (no V yet), NOT_SPD, DEVICE. */
nmf_status nmf_enforce(nmf_handle* h, int32_t mode, int64_t t_u, int64_t t_v);

/* Documents per topic and label, for the clustering accuracy of Eq. (acc)
 * (Section 3.2): counts[c * n_labels + l] (k x n_labels, host) = the number
 * of documents with labels[d] == l that store an entry in column c of V (a
 * document belongs to a topic when that entry is nonzero).  labels: m
 * int32 in [0, n_labels) (others are skipped), host or device;
 * 1 <= n_labels <= 256.  Synchronizes.  Errors: INVALID_ARG, STATE (no V). */
nmf_status nmf_topic_counts(nmf_handle* h, const int32_t* labels, int32_t n_labels, int64_t* counts);

/* Clustering accuracy of Eq. (acc) (Section 3.2) of every topic of the
 * current V: acc[c] (k doubles, host) for the documents storing an entry in
 * column c, labelled by labels[d] in [0, n_labels) as in nmf_topic_counts
 * (the counts come from the same device kernel).  With S the topic's
 * same-label document pairs, n_D its documents, n_J = n_labels and
 * q, r = n_D div n_J, n_D mod n_J:
 *   acc = (S - alpha) / (beta - alpha),
 *   alpha = q (n_J (q - 1) / 2 + r)   (pairs of the most even spread),
 *   beta  = n_D (n_D - 1) / 2         (pairs of a single-label topic),
 * evaluated exactly in 64-bit integers up to the final division; a topic
 * with at most one document, or n_J = 1, scores 1.  Synchronizes.
 * Errors: as nmf_topic_counts. */
nmf_status nmf_topic_accuracy(nmf_handle* h, const int32_t* labels, int32_t n_labels, double* acc);

/* The arithmetic of nmf_topic_accuracy on counts the caller holds (host,
 * k x n_labels, row-major, counts[c * n_labels + l] >= 0): acc[c] for
 * c < k (host).  Needs no handle and no device.  Errors: INVALID_ARG
 * (NULL pointer, k < 1, n_labels < 1, a negative count). */
nmf_status nmf_accuracy_from_counts(const int64_t* counts, int32_t k, int32_t n_labels, double* acc);

/* Read a tuning parameter into *value.  Errors: INVALID_ARG. */
nmf_status nmf_get_param(nmf_handle* h, int32_t param, int64_t* value);

/* Message for the last error on this handle (or of the last failed
 * nmf_create when h is NULL).  Never NULL. */
const char* nmf_last_error(const nmf_handle* h);

/* Release the handle (host memory only; the workspace stays the caller's).
 * Waits for the handle's stream.  NULL is allowed. */
void nmf_destroy(nmf_handle* h);

/* ---- Batched solving: many independent problems advanced together -------
 *
 * Each problem is the method above (Algorithm 2 with the per-column rule of
 * Section 4) on its own A, U0, k and t; problems may differ in every size.
 * A batch owns one handle per problem (reachable with nmf_batch_problem for
 * errors, histories and factors) and advances all of them the same number of
 * iterations.  Four ways to run the same iterations, all producing bitwise
 * identical factors:
 *   NMF_BATCH_LOOP         every problem's own launches, problem after problem
 *                          (what a caller looping over nmf_als_step does);
 *   NMF_BATCH_LOOP_GRAPH   the same launches captured once as a HIP graph of
 *                          two iterations and replayed;
 *   NMF_BATCH_FUSED        one launch per stage for all problems: every block
 *                          of the launch serves one (problem, block) pair of
 *                          that problem's own grid;
 *   NMF_BATCH_FUSED_GRAPH  the fused launches captured as a HIP graph of two
 *                          iterations and replayed. */
typedef struct nmf_batch nmf_batch;

enum { NMF_BATCH_LOOP = 0, NMF_BATCH_LOOP_GRAPH = 1, NMF_BATCH_FUSED = 2, NMF_BATCH_FUSED_GRAPH = 3 };

/* Device workspace bytes for a batch of `count` problems (cfgs[i], nnz[i]):
 * the problems' own workspaces plus the fused launch tables.
 * Errors: INVALID_ARG, UNSUPPORTED (as nmf_workspace_size, per problem). */
nmf_status nmf_batch_workspace_size(int32_t count, const nmf_config* cfgs, const int64_t* nnz, size_t* bytes);

/* Create a batch.  Arrays of `count` entries: cfgs, a_rowptr, a_col, a_val,
 * nnz and u0 are as the arguments of nmf_create for each problem (host or
 * device pointers; V0 is not taken).  workspace: device, 256-byte aligned, at
 * least nmf_batch_workspace_size bytes, owned by the caller and untouched
 * after nmf_batch_destroy.  hip_stream: the stream every problem runs on; the
 * graph modes need a stream that can be captured, so with NULL the batch
 * creates (and later destroys) a stream of its own.  *out receives the
 * batch.  Errors: those of nmf_create (the first failing problem's, with its
 * index in the message), WORKSPACE. */
nmf_status nmf_batch_create(int32_t count, const nmf_config* cfgs, const int64_t* const* a_rowptr,
                            const int32_t* const* a_col, const void* const* a_val, const int64_t* nnz,
                            const void* const* u0, void* workspace, size_t ws_bytes, void* hip_stream,
                            nmf_batch** out);

/* Enqueue `iters` ALS iterations of every problem, run as `how`
 * (NMF_BATCH_*).  Asynchronous.  A problem whose device status turns sticky
 * stops advancing (its kernels return at once) while the others continue.
 * The first graph-mode call captures the graph (and so takes longer).
 * Errors: INVALID_ARG (iters < 0, unknown how), DEVICE, STATE (a graph or
 * fused mode after some problem was stepped on its own handle: the problems'
 * iterates are out of step; NMF_BATCH_LOOP still runs). */
nmf_status nmf_batch_step(nmf_batch* b, int32_t iters, int32_t how);

/* Set a tuning parameter (as nmf_set_param) of problem i, or of every
 * problem for i = -1, and record the fused launches again (captured graphs
 * are dropped and captured anew by the next graph-mode call).  Synchronizes.
 * Errors: INVALID_ARG, those of nmf_set_param (with the problem's index). */
nmf_status nmf_batch_set_param(nmf_batch* b, int32_t i, int32_t param, int64_t value);

/* Autotuner of the fused form: for each half-step in turn (V, then U), tries
 * a fixed list of SpMM forms (step form, entry-by-entry threshold, waves per
 * block) on all problems at once, each for 1 + `iters` fused iterations
 * timed with HIP events on the batch's stream, and keeps the fastest.  The
 * trials are real iterations: every problem advances 16 * (1 + iters)
 * iterations.  chosen (may be NULL) receives 6 ints: {wide, entry threshold,
 * waves} of the V half, then of the U half.  Synchronizes.
 * Errors: INVALID_ARG (iters < 1), STATE (problems out of step), DEVICE. */
nmf_status nmf_batch_tune(nmf_batch* b, int32_t iters, int32_t* chosen);

/* Wait for the batch, then for every problem i: E[i] = its relative error
 * (as nmf_error) and status[i] = its status (NMF_OK or the sticky error).
 * Either array may be NULL.  Returns NMF_OK when every problem is OK, else
 * the first problem's error. */
nmf_status nmf_batch_errors(nmf_batch* b, double* E, int32_t* status);

/* The handle of problem i (owned by the batch: do not destroy it), or NULL. */
nmf_handle* nmf_batch_problem(nmf_batch* b, int32_t i);

/* Message for the last error of the batch (or of the last failed
 * nmf_batch_create when b is NULL).  Never NULL. */
const char* nmf_batch_last_error(const nmf_batch* b);

/* Release the batch and its problems' handles (host memory and the batch's
 * own stream and graphs).  NULL is allowed. */
void nmf_batch_destroy(nmf_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* NMF_H */
