/*
 * coreals.h -- C ABI of the MI355X (gfx950) library for core-elements
 * subsampled alternating least squares.
 *
 * Method: Xue, Li, Zhang and Meng, "Core-elements Subsampling for Alternating
 * Least Squares".  Problem statement in Section 2.1: a rating matrix R with
 * observed index set I, rank n_f, factor matrices U (n_u x n_f) and
 * M (n_m x n_f), and the weighted-lambda objective
 *     f(U, M) = sum_I (r_ij - u_i m_j^T)^2 + lambda (sum_i n_i |u_i|^2 + sum_j n_j |m_j|^2).
 * Core-ALS (Algorithm 2) alternates two half-sweeps.  Every row regression
 * builds a sparse sketch X* of its design matrix X with CES (Algorithm 1:
 * per column keep the floor(n_i r) entries of largest magnitude) and solves
 *     (X*^T X + lambda n_i E) u = X*^T y            (eq. core_ui / core_mj).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless the comment says (host).
 *  - The caller owns every array, including the workspace; the library owns
 *    only the opaque context (host memory).
 *  - Every call is enqueued on the stream given in als_problem.stream
 *    (a hipStream_t; NULL means the default stream).  Calls marked "syncs"
 *    wait for that stream before returning.
 *  - Calls return als_status and never abort.  als_last_error() describes the
 *    most recent failure on a context.
 *  - A context is not thread-safe; use one context per stream.
 *  - Index layout: CSR row_ptr int64[n_rows+1] starting at 0; col_idx int32,
 *    strictly increasing inside a row; val float32.  Factor matrices are
 *    float32, row-major, row stride n_f, and must not alias each other.
 */
#ifndef CORE_ALS_H
#define CORE_ALS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct als_ctx als_ctx;

typedef enum {
    ALS_OK = 0,
    ALS_E_ARG = 1,     /* bad size, rate, precision or NULL pointer          */
    ALS_E_INDEX = 2,   /* row_ptr not monotone, column out of range, repeated
                          or unsorted column inside a row                      */
    ALS_E_VALUE = 3,   /* NaN or Inf among the ratings (ALS_VALIDATE only)    */
    ALS_E_NOMEM = 4,   /* workspace or output buffer too small                */
    ALS_E_DEVICE = 5,  /* a HIP runtime error                                 */
    ALS_E_STATE = 6    /* call not valid on this context                      */
} als_status;

typedef enum {
    ALS_PREC_FP32 = 0,            /* FP32 Gram (heavy rows: FP32 products from
                                     an exact three-way bf16 split on bf16
                                     MFMA tiles, FP32 accumulation), FP32
                                     solve                                    */
    ALS_PREC_BF16_IR = 1,         /* heavy rows: BF16 MFMA Gram (FP32 accumulate),
                                     FP32 LU, one refinement step with an FP32
                                     residual; light rows: FP32 Gram          */
    ALS_PREC_BF16_IR_FP64RES = 2, /* as above, refinement residual in FP64    */
    ALS_PREC_AUTO = 3             /* BF16 + refinement with a per-row choice
                                     from the condition estimate kappa =
                                     |A|_inf |A^-1 e|_inf / |e|_inf (one extra
                                     solve with the LU factors): kappa > 2^8,
                                     the row's Gram is built again with FP32
                                     products; lambda < 1e-3 and kappa > 2^10,
                                     its refinement residual is FP64        */
} als_precision;

#define ALS_VALIDATE 1u   /* check ratings for NaN/Inf in als_init */
#define ALS_USERS_ONLY 2u /* users side only: no column view is built, and
                             half_sweep_items, core_select(side 1) and objective
                             return ALS_E_STATE (contexts of new users to fold
                             in, see foldin_answer) */
#define ALS_FAST_VARIANT 8u /* the fast variant of Core-ALS (Section 3, the
                               paragraph after Algorithm 2): before each
                               half-sweep CES is applied once to the whole
                               factor matrix of the other side (rate r, budget
                               floor(n_other r) per column), and every row
                               regresses on that global sketch: A = X*^T X +
                               lambda n_i E with X* the row's rows of the
                               sketch, a singular A replaced by eq. (U).  The
                               number of kept entries per row then only follows
                               r on average.  Needs n_f <= 64, ALS_PREC_FP32,
                               both sides (not ALS_USERS_ONLY); core_select is
                               replaced by core_select_global */
#define ALS_UNIF 16u /* UNIF, the uniform-subsampling comparator of Section 5:
                        each regression draws s = min(n_i, max(min_keep,
                        floor(n_i r))) of its entries uniformly without
                        replacement (the s smallest keys h(seed, row, col) =
                        upper 32 bits of splitmix64 at seed * 0x9E3779B97F4A7C15
                        + row * n_cols + col, ties by position; n_cols = rows
                        of the other factor matrix) and solves
                        (X_S^T X_S + lambda s E) u = X_S^T y_S.  The seed is
                        set with als_set_sample_seed (default 0).  Needs
                        n_f <= 64, ALS_PREC_FP32, not ALS_FAST_VARIANT;
                        n_singular_fallback counts singular sample systems
                        (answered with u = 0) */
#define ALS_IMPLICIT 32u /* implicit-feedback Core-ALS (Section 3, last
                            paragraph; the form is a reading, the paper's
                            appendix is not in its text): the ratings are
                            confidences, every observed entry a preference 1
                            with confidence 1 + alpha r, every other entry a
                            preference 0 with confidence 1 (Hu, Koren and
                            Volinsky); a row solves
                            (Y^T Y + X*^T W X + lambda E) u = X*^T (1 + alpha r)
                            with Y the whole other factor matrix, X its rows at
                            the row's entries, W = diag(alpha r), X* = CES(X)
                            (Algorithm 1).  r = 1 is implicit ALS.  Uses
                            als_problem.alpha >= 0; needs n_f <= 64,
                            ALS_PREC_FP32, not ALS_FAST_VARIANT / ALS_UNIF;
                            objective returns ALS_E_STATE */
#define ALS_GENERIC_GATHERS 4u /* heavy-row kernels gather with 64-bit addresses
                                 even where 32-bit buffer offsets would do (the
                                 path taken for factor matrices of 2^24 rows or
                                 2^31 bytes and more; slower, for tests) */

typedef struct {
    int64_t n_u, n_m, nnz;
    int32_t n_f;                 /* 1 <= n_f <= 128; ranks above 64 solve every
                                    row with a workgroup (heavy-row schedule),
                                    and foldin_answer needs n_f <= 64           */
    const int64_t *row_ptr;      /* CSR of R (users x items), device          */
    const int32_t *col_idx;
    const float *val;
    double lambda;               /* >= 0; row i gets lambda * n_i on the diagonal */
    uint32_t budget_num;         /* subsampling rate r = budget_num / budget_den,   */
    uint32_t budget_den;         /* 0 < r <= 1; r = 1 is full-data ALS              */
    int32_t min_keep;            /* s_i = min(n_i, max(min_keep, floor(n_i r)))     */
    int32_t precision;           /* als_precision                                   */
    uint32_t flags;              /* ALS_VALIDATE | ALS_USERS_ONLY | ALS_GENERIC_GATHERS */
    void *stream;                /* hipStream_t                                     */
    void *workspace;             /* device buffer, at least als_workspace_size bytes */
    size_t workspace_bytes;
    int32_t heavy_min_degree;    /* schedule: rows of higher degree (or budget > 32)
                                    are split across workgroups; 0 = default 1024 */
    int32_t heavy_chunk;         /* entries per partial Gram of such rows; 0 = 1024 */
    int32_t heavy_pair_cap;      /* partial systems kept in scratch at once (sizes the
                                    workspace); 0 = 65536 (8192 for n_f > 64) */
    int32_t light_blocks;        /* grid of the persistent light-row kernels, whose
                                    wavefronts take rows from an atomic counter;
                                    0 = one row per wavefront */
    const int64_t *col_ptr;      /* optional column view (CSC) of the same R, device:
                                    col_ptr int64[n_m+1], row_idx int32[nnz] strictly
                                    increasing inside a column, val_t float32[nnz];
                                    all NULL = built by als_init in the workspace.
                                    Checked like the CSR (not against it); kept by
                                    pointer until als_destroy                       */
    const int32_t *row_idx;
    const float *val_t;
    double alpha;                /* ALS_IMPLICIT: confidence 1 + alpha r per rating */
} als_problem;

typedef struct {
    int64_t n_empty;             /* rows with no observed entry: output row is 0   */
    int64_t n_singular_fallback; /* core systems with a pivot below n_f 2^-23 max|A|,
                                    replaced by the full-data update eq. (U)      */
    int64_t n_fp64_residual;     /* rows refined with an FP64 residual            */
    int64_t n_rows;              /* rows solved in this half-sweep                */
    int64_t n_fp32_gram;         /* ALS_PREC_AUTO: rows whose Gram was built again
                                    with FP32 products (condition estimate)       */
    double max_rel_residual;     /* BF16 modes: largest relative residual
                                    |b - A u0| / |b| of a refined row's first
                                    solution u0 (A u = b its system); 0 when no
                                    row is refined                                */
    int64_t n_select_hinted;     /* heavy rows whose selection found each column's
                                    16-bit threshold in one counting pass over a
                                    window around the same row's threshold of the
                                    previous half-sweep of this side (the cuts are
                                    exact either way)                             */
    int64_t n_pivoted;           /* rows whose elimination without row exchanges
                                    was rejected (a small pivot, an entry grown
                                    beyond 4 max|A| or a multiplier above 4) and
                                    that were solved again with partial pivoting:
                                    light core rows and heavy rows (the n x n
                                    systems of rows of at most 32 entries retry
                                    the same way, uncounted)                      */
} als_sweep_stats;

typedef struct {
    double f;      /* objective of Section 2.1                                    */
    double sse;    /* sum of squared residuals over I                              */
    double rmse;   /* sqrt(sse / nnz)                                               */
    double remse;  /* sqrt(sse) / sqrt(sum r^2)   (ReMSE, Section 5.1)              */
} als_objective;

/* Bytes of device workspace als_init needs for this problem (host only, no
 * device call).  Returns 0 if the problem sizes are invalid. */
size_t als_workspace_size(const als_problem *p);

/* Validate R on the device, build its column view (CSC, rows ascending inside
 * a column) in the workspace, compute degrees n_i, budgets s_i and the degree
 * classes that schedule the half-sweeps.  The CSR arrays must stay alive and
 * unchanged until als_destroy.  Syncs once.  Errors: ALS_E_ARG, ALS_E_INDEX,
 * ALS_E_VALUE, ALS_E_NOMEM (workspace too small), ALS_E_DEVICE. */
als_status als_init(const als_problem *p, als_ctx **out);

/* Half-sweep over users (Algorithm 2, first loop; eq. core_ui): for every user
 * i, X = rows of M indexed by the user's observed items, y = the user's
 * ratings; CES on X, then U[i] = (X*^T X + lambda n_i E)^-1 X*^T y.
 * M: [n_m * n_f] input; U: [n_u * n_f] output.  If st is non-NULL (host) the
 * call syncs and fills the per-row event counts; otherwise it is fully
 * asynchronous. */
als_status half_sweep_users(als_ctx *c, const float *M, float *U, als_sweep_stats *st);

/* Half-sweep over items (Algorithm 2, second loop; eq. core_mj), the same
 * regression over the columns of R with U as the design side.
 * U: [n_u * n_f] input; M: [n_m * n_f] output. */
als_status half_sweep_items(als_ctx *c, const float *U, float *M, als_sweep_stats *st);

/* Half-sweep of side 0 (users, other = M, out = U) or side 1 (items,
 * other = U, out = M) exactly as half_sweep_users / half_sweep_items, for
 * callers that cannot allocate device memory (code under stream capture,
 * serving loops, hosts that forbid it): the call's scratch (event counters,
 * row-queue counters, heavy-row partial systems and refinement residuals)
 * lives in a fixed array of the library in device memory,
 * half_sweep_noalloc_scratch_bytes() bytes per GPU (about 18 MB), held from
 * the first call on that GPU until the process ends, instead of in the
 * context's workspace.  It calls no allocator.  The context must have been
 * created with heavy_pair_cap <= half_sweep_noalloc_pair_cap() (1024);
 * ALS_E_ARG otherwise, and for contexts created with ALS_FAST_VARIANT,
 * ALS_UNIF or ALS_IMPLICIT (their selection state and Gram stay in the
 * workspace).  Results are identical to the workspace entry points'.
 * The array keeps the last call's contents and every call on a GPU shares
 * it: calls that overlap in time on one GPU (several streams or threads)
 * race.  Never captured into the context's graphs; no profiling marks.  st
 * as for half_sweep_users. */
als_status half_sweep_noalloc(als_ctx *c, int side, const float *other, float *out, als_sweep_stats *st);
size_t half_sweep_noalloc_scratch_bytes(void);
int64_t half_sweep_noalloc_pair_cap(void);

/* Number of positions core_select writes for rows [row_begin, row_end) of one
 * side: sum over rows of n_f * s_i.  side 0 = users (rows of R), 1 = items
 * (columns of R).  *count is (host).  Syncs. */
als_status core_select_count(als_ctx *c, int side, int64_t row_begin, int64_t row_end,
                             int64_t *count);

/* CES of Algorithm 1 for rows [row_begin, row_end) of one side, with `other`
 * the opposite factor matrix (M for side 0, U for side 1).
 * sel_ptr: [row_end - row_begin + 1] int64 output, sel_ptr[t] = offset of
 * row row_begin + t.  sel_pos: output of capacity sel_cap int32; row t,
 * column a occupies sel_pos[sel_ptr[t] + a*s .. + s), the s kept positions
 * (0-based offsets into the row's observed entries) in ascending order.
 * Ties in |x| keep the smaller position.  ALS_E_NOMEM if sel_cap is below
 * core_select_count.  Asynchronous. */
als_status core_select(als_ctx *c, int side, const float *other, int64_t row_begin,
                       int64_t row_end, int64_t *sel_ptr, int32_t *sel_pos, int64_t sel_cap);

/* The fast variant's global sketch (ALS_FAST_VARIANT contexts): CES of
 * Algorithm 1 on the whole matrix `other` (M for side 0, U for side 1; n_other
 * x n_f) with budget s = min(n_other, max(min_keep, floor(n_other r))) per
 * column.  Writes the cut of column a: T[a], K[a] (device int32 [n_f]); entry
 * (j, a) is kept iff bits(|other[j][a]|) > T[a], or equal and j <= K[a]
 * (ties keep the smaller row j).  Asynchronous.  ALS_E_STATE on contexts
 * without ALS_FAST_VARIANT. */
als_status core_select_global(als_ctx *c, int side, const float *other, int32_t *T, int32_t *K);

/* Objective of Section 2.1 at (U, M), with SSE, RMSE and ReMSE (Section 5.1),
 * accumulated in FP64 in a fixed order (deterministic).  out is (host).  Syncs. */
als_status objective(als_ctx *c, const float *U, const float *M, als_objective *out);

/* Kernel timing for measurement.  After als_profile_begin, every half-sweep
 * records a pair of HIP events around each kernel (group) it launches (on the
 * problem's stream; no synchronisation is added).  als_profile_end syncs and
 * fills (host) ms[side*12 + k] with the summed time and launches[side*12 + k]
 * with the number of launches since als_profile_begin.  side 0 = users,
 * 1 = items; k = 0: light full-data rows, 1..6: light rows with insertion
 * networks of capacity 1, 2, 4, 8, 16, 32, 7: heavy-row selection, 8: heavy-row
 * Gram chunks, 9: heavy-row solves, 10: refinement residuals, 11: refinement
 * solves.  Either array may be NULL.  Profiling then stops. */
als_status als_profile_begin(als_ctx *c);
als_status als_profile_end(als_ctx *c, double *ms, int64_t *launches);

/* Seed of the UNIF draws of the following half-sweeps (ALS_UNIF contexts;
 * no effect otherwise).  No device call. */
als_status als_set_sample_seed(als_ctx *c, uint64_t seed);

/* Capture each half-sweep into a HIP graph on its first call and replay the
 * graph on later calls with the same factor pointers (a call with other
 * pointers captures a new graph).  Needs a non-default stream (ALS_E_STATE
 * otherwise).  Profiling calls are never captured. */
als_status als_use_graphs(als_ctx *c, int enable);

/* Row counts of the degree classes (host out[side*8 + cls]); no device call. */
als_status als_class_counts(const als_ctx *c, int64_t *out);

/* Release the context (host memory only; the caller frees its buffers). */
void als_destroy(als_ctx *c);

/* ------------------------------------------------------------------------
 * Learned fold-in of new users.  Beyond the method itself: a small network
 * answers a new user (ratings on the trained items, M frozen) from the
 * embedding bag b = (1/d) sum_k r_k M[j_k] of its d ratings:
 *     h1 = GELU(W1 b + c1), h2 = GELU(W2 h1 + c2), u = W3 h2 + c3,
 * GELU(x) = x Phi(x).  It is trained on factor rows that ALS produced, and an
 * answer is kept only when the relative residual |b_i - A_i u| / |b_i| of the
 * user's own regression (A_i u = b_i: eq. core_ui at the context's rate,
 * eq. (U) when r = 1) is within a tolerance; otherwise that regression is
 * solved exactly (one direct solve, as in a users half-sweep).
 *
 * Parameters are one float vector of foldin_param_count(n_f, hidden) entries:
 * W1 [hidden x n_f], c1 [hidden], W2 [hidden x hidden], c2 [hidden],
 * W3 [n_f x hidden], c3 [n_f], each row-major.  FP32 master weights; matrix
 * products on MFMA with bf16 operands and FP32 accumulation (FOLDIN_BF16) or
 * FP32 operands (FOLDIN_FP32).  All calls run on cfg.stream (foldin_answer:
 * on the query context's stream) and are asynchronous unless marked "syncs".
 * ---------------------------------------------------------------------- */
typedef struct foldin_model foldin_model;

typedef enum { FOLDIN_BF16 = 0, FOLDIN_FP32 = 1 } foldin_precision;

typedef struct {
    int32_t n_f;            /* input and output width, 1..64                    */
    int32_t hidden;         /* hidden width, 1..1024                           */
    int32_t max_batch;      /* most rows per forward / gradient batch, 1..2^20 */
    int32_t precision;      /* foldin_precision                                 */
    int64_t max_train_rows; /* most rows foldin_train may shuffle (sizes the workspace) */
    float lr, beta1, beta2, eps, weight_decay;   /* AdamW (decoupled decay)     */
    void *stream;           /* hipStream_t                                      */
    void *workspace;        /* device buffer of foldin_workspace_size bytes; holds the
                               weights, AdamW moments, activations and gradients */
    size_t workspace_bytes;
} foldin_cfg;

typedef struct {
    int64_t n_rows;              /* users answered                                 */
    int64_t n_mlp;               /* answers of the network kept                    */
    int64_t n_exact;             /* users solved exactly (residual above tol, or no
                                    ratings: answer 0)                             */
    int64_t n_empty;             /* users without ratings                          */
    int64_t n_singular_fallback; /* exact solves whose core system was singular and
                                    used the full-data update eq. (U) instead      */
} foldin_answer_stats;

/* Number of parameters (0 for invalid sizes).  Host only. */
int64_t foldin_param_count(int32_t n_f, int32_t hidden);

/* Workspace bytes for cfg (0 if cfg is invalid).  Host only. */
size_t foldin_workspace_size(const foldin_cfg *cfg);

/* Create a model in cfg->workspace with initial weights `params` (device,
 * copied) and zero AdamW moments.  ALS_E_ARG for invalid sizes, ALS_E_NOMEM if
 * the workspace is too small. */
als_status foldin_create(const foldin_cfg *cfg, const float *params, foldin_model **out);

/* Copy the current weights to params (device), or replace them (moments and
 * step count reset). */
als_status foldin_get_params(foldin_model *m, float *params);
als_status foldin_set_params(foldin_model *m, const float *params);

/* Network answers for n users: U_out[b] for user rows[b] (rows: device int32
 * [n], or NULL for users 0..n-1) of the CSR (ptr, items, vals) over the items
 * of M [n_items x n_f].  U_out: device [n * n_f].  The CSR and rows are not
 * checked here: they must be valid as als_init checks them (monotone ptr,
 * item indices below n_items, row ids inside the CSR). */
als_status foldin_forward(foldin_model *m, const float *M, const int64_t *ptr, const int32_t *items,
                          const float *vals, const int32_t *rows, int64_t n, float *U_out);

/* Forward and backward pass of one batch (1..max_batch rows, as in
 * foldin_forward) against target rows target[rows[b]] ([* x n_f], device):
 * loss = mean over the batch and the n_f outputs of (u - target)^2.  Writes the
 * gradient of the loss (device [param_count], optional) and the loss (device
 * float, optional). */
als_status foldin_grad(foldin_model *m, const float *M, const int64_t *ptr, const int32_t *items,
                       const float *vals, const int32_t *rows, int64_t n, const float *target, float *grad,
                       float *loss);

/* One AdamW step with gradient grad (device [param_count]), or with the
 * gradient of the last foldin_grad when grad is NULL. */
als_status foldin_adamw(foldin_model *m, const float *grad);

/* Train for `epochs` passes over rows 0..n_rows-1 of the CSR, in batches of
 * `batch` rows shuffled per epoch by a splitmix64 stream seeded with `seed`;
 * one AdamW step per batch.  loss_per_epoch (host [epochs], optional): mean
 * batch loss of each epoch.  Syncs once per epoch. */
als_status foldin_train(foldin_model *m, const float *M, const int64_t *ptr, const int32_t *items,
                        const float *vals, int64_t n_rows, const float *target, int32_t epochs, int32_t batch,
                        uint64_t seed, float *loss_per_epoch);

/* Answer the users of the query context q (its CSR holds the new users'
 * ratings over the n_m items of M; create it with ALS_USERS_ONLY and the
 * lambda, rate and precision the exact regressions should use).  Writes
 * U_new [n_u x n_f] (device): the network's answer where the relative
 * residual rho[i] (device float [n_u]) of user i's regression is <= tol, the
 * exact solution otherwise; path[i] (device int32 [n_u]) = 0 for a kept
 * answer, 1 for an exact one.  st (host, optional) makes the call sync. */
als_status foldin_answer(als_ctx *q, foldin_model *m, const float *M, double tol, float *U_new, int32_t *path,
                         float *rho, foldin_answer_stats *st);

/* Release the model (host memory only). */
void foldin_destroy(foldin_model *m);

/* Message of the last failure on m. */
const char *foldin_last_error(const foldin_model *m);

/* Message of the last failure on c (or of the last failed als_init when c is
 * NULL).  Valid until the next call on the same context. */
const char *als_last_error(const als_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* CORE_ALS_H */
