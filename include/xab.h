/*
 * xab: auto-tuned CSR sparse matrix-vector products and Krylov drivers for
 * AMD MI355X (gfx950).  C ABI.
 *
 * The operations follow the problem statement of Katagiri et al., "Xabclib:
 * a fully auto-tuned sparse iterative solver":
 *   - SpMV y = A x on a CRS matrix, with several thread layouts chosen at
 *     run time by measuring them (section 3.1, section 3.2.2): the
 *     row-based decomposition, the non-zero-elements based (load balanced)
 *     decomposition and the branchless segmented scan for unsymmetric A;
 *     the symmetric product from one stored triangle with zero-element
 *     omission in the transpose-part reduction for symmetric A;
 *   - the linear-solve drivers restarted GMRES(m) and BiCGStab (section 2.2)
 *     under the accuracy policy's true-residual check (section 3.3.2).
 * The library adds a learned cost model to the selector, FP32-value SpMV
 * inside GMRES with FP64 iterative refinement, and a batched BiCGStab over
 * many independent systems.
 *
 * Conventions
 *   - Pointers named d_* are DEVICE memory, h_* HOST memory.  Every d_*
 *     argument is owned by the caller and borrowed: it must stay valid and
 *     unmodified while any matrix, plan or batch that references it exists.
 *   - Matrix arrays (rowptr, colind, values) must be 16-byte aligned.
 *   - Indices are int32 (row pointers, column indices); nnz < 2^31.
 *   - SpMV calls are queued on the context's stream and return without
 *     waiting.  Calls documented as "synchronous" wait for the stream.
 *   - A context is not thread-safe: use one context per host thread/stream.
 *   - Every call returns an int status.  0 is success.  Negative codes are
 *     caller errors: nothing was computed and the outputs are unspecified.
 *     Positive codes mean the call computed a result but with the numerical
 *     outcome named (not converged, breakdown, time limit).  No caller
 *     memory is ever freed by the library.
 */
#ifndef XAB_H
#define XAB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define XAB_OK 0
#define XAB_E_NULL (-1)        /* a required pointer is null */
#define XAB_E_SHAPE (-2)       /* negative or inconsistent sizes */
#define XAB_E_DTYPE (-3)       /* unsupported precision combination */
#define XAB_E_STRUCT (-4)      /* invalid CSR (rowptr, column range, upper entry in lower storage) */
#define XAB_E_ALIAS (-5)       /* input and output vectors overlap */
#define XAB_E_UNSUPPORTED (-6) /* variant not applicable to this matrix or parameters */
#define XAB_E_NOMEM (-7)       /* device allocation failed */
#define XAB_E_DEVICE (-8)      /* HIP runtime error; see xab_last_error */
#define XAB_E_ALIGN (-9)       /* matrix array not 16-byte aligned */
#define XAB_NOT_CONVERGED 1    /* iteration limit reached */
#define XAB_BREAKDOWN 2        /* a Krylov recurrence divided by zero */
#define XAB_TIME_LIMIT 3       /* wall-clock limit reached (the policy's MAXTIME) */

typedef struct xab_ctx xab_ctx;
typedef struct xab_matrix xab_matrix;
typedef struct xab_plan xab_plan;
typedef struct xab_batch xab_batch;

typedef enum { XAB_F64 = 0, XAB_F32 = 1 } xab_dtype;

/* Numerical computation policy (section 2.3): TIME picks the fastest
 * measured implementation; STABLE runs without auto-tuning (fixed default);
 * LEARNED uses the trained cost model instead of timing; MEMORY sets
 * arguments for the least device memory: the selector keeps to the
 * implementations whose plans hold the fewest bytes (see xab_select), and
 * on a context whose default policy is MEMORY the solvers do not grow the
 * restart length (the basis keeps its starting size); ACCURACY selects as
 * TIME does, and on a context whose default policy is ACCURACY GMRES
 * follows the accuracy policy's orthogonalisation rule and fault-convergence
 * retry (XAB_ORTHO_POLICY, section 3.3.2) whatever opts->ortho asks, and
 * the batched BiCGStab reruns systems whose true residual misses tol. */
typedef enum { XAB_TIME = 0, XAB_STABLE = 1, XAB_LEARNED = 2, XAB_MEMORY = 3, XAB_ACCURACY = 4 } xab_policy;

/* SpMV implementations (section 3.2.2 candidate list):
 *   XAB_ROW        row-based decomposition, equal rows per workgroup,
 *                  lanes_per_row lanes cooperating on a row
 *   XAB_NNZ        non-zero elements based decomposition: whole rows,
 *                  about tile_nnz entries per workgroup
 *   XAB_BSS        branchless segmented scan over the entry stream,
 *                  256 * j_per_lane entries per workgroup
 *   XAB_SYM_S3     symmetric, lower storage, zero-element omission in the
 *                  transpose reduction (column blocks of col_block rows);
 *                  reproducible bit for bit (every addition in an order
 *                  fixed by the plan).  When the padding stays within a
 *                  quarter of the entries and no row exceeds 4096 entries
 *                  the plan keeps a sliced copy of the matrix (chunks of
 *                  64 rows, one lane per row) and values changed after
 *                  plan creation are not seen; otherwise it walks the
 *                  caller's CSR entries.  Fewer than 2^30 - 1 rows.
 *   XAB_SYM_ATOMIC symmetric, lower storage, transpose part by device
 *                  atomics (baseline; not bitwise reproducible)
 *   XAB_XCB        column-blocked segmented scan: the plan copies the
 *                  matrix into 8 column blocks (one per XCD of the MI355X)
 *                  so each block's slice of x stays in one XCD's L2; each
 *                  block is scanned with 256 * j_per_lane entries per
 *                  workgroup and the 8 partial products are summed in
 *                  block order.  The plan owns the copy: values changed
 *                  after plan creation are not seen.
 *   XAB_SELL       sliced ELLPACK with a sorting window (SELL-C-sigma, a
 *                  format the paper names as future work, section 5):
 *                  inside windows of tile_rows rows the rows are ordered
 *                  longest first, cut into chunks of 64 (one wave) and each
 *                  chunk is stored column-major, padded to its longest row;
 *                  one lane sums one row.  The plan owns the padded copy.
 *                  XAB_E_UNSUPPORTED when a row is longer than 4096 or the
 *                  padded size would exceed twice the entries plus one
 *                  chunk of the longest row.
 *   XAB_BCSR       block CSR with 4 x 4 blocks (another future-work format
 *                  of section 5): block row R covers rows 4R .. 4R+3, its
 *                  blocks are the distinct column blocks c / 4 of its
 *                  entries, each stored as 16 values (row-major, zeros
 *                  where no entry, duplicates summed) plus a mask of the
 *                  stored positions; one lane sums one block row.  The plan
 *                  owns the copy.  XAB_E_UNSUPPORTED when a block row has
 *                  more than 4096 entries or the blocks would hold more
 *                  than twice the entries. */
typedef enum {
    XAB_ROW = 0,
    XAB_NNZ = 1,
    XAB_BSS = 2,
    XAB_SYM_S3 = 3,
    XAB_SYM_ATOMIC = 4,
    XAB_XCB = 5,
    XAB_SELL = 6,
    XAB_BCSR = 7
} xab_variant;

typedef struct {
    int32_t lanes_per_row; /* ROW, SYM_ATOMIC: 1, 2, 4, ..., 64 */
    int32_t tile_nnz;      /* NNZ, SYM_S3: target entries per tile (>= 256); SYM_S3 with
                              tile_rows >= 256 moves each tile boundary to the nearest
                              multiple of 256 rows (whole rounds of the four-wave walk) */
    int32_t j_per_lane;    /* BSS, XCB: entries per lane, a power of two in 1..32; XCB also
                              takes 0: the largest of 4, 8, 16, 32 that leaves at least
                              4096 tiles of 256 * j_per_lane entries (xab_plan_info reports it);
                              FP32 values then take the same rule capped at 16, with their own
                              copy of the columns when that differs */
    int32_t col_block;     /* SYM_S3: column block size C of the touch map (power of two) */
    int32_t tile_rows;     /* SYM_S3: maximum rows per tile (<= 2048); SELL: sorting window
                              (a multiple of 64, at most 1024) */
    int32_t xcb_slices;    /* XCB: column slices walked one after another, each cut into 8
                              blocks (one per XCD), a power of two in 1..64; 0: from the size,
                              the fewest that keep every block under 262,144 columns (2 MB of
                              FP64 x, half an XCD's L2) */
} xab_params;

/* Matrix flags */
#define XAB_GENERAL 0u
#define XAB_SYM_LOWER 1u   /* symmetric; only entries with col <= row are stored */
#define XAB_TRUST_INPUT 2u /* skip the structural validation pass */
#define XAB_BATCH_TILES 4u /* xab_batch_csr: segmented-scan tiles only, no sliced ELLPACK copy */

/* Selector classes: fixed (variant, params) pairs, the action space of the
 * selector.  0..8 and 12..14 apply to general matrices, 9..11 to
 * XAB_SYM_LOWER. */
#define XAB_NCLASSES 15
int xab_class_params(int32_t k, xab_variant *variant, xab_params *params);

typedef struct {
    int32_t device;                         /* HIP device ordinal; -1 = current */
    void *stream;                           /* hipStream_t to queue on; NULL = default stream */
    void *(*alloc)(size_t bytes, void *user); /* optional device allocator */
    void (*free)(void *ptr, void *user);      /* optional, pairs with alloc */
    void *user;
    int32_t policy;                         /* default xab_policy */
} xab_init_opts;

/* Create a context: device, stream, allocator and policy defaults (the
 * paper's initialisation call that sets library defaults, Table 1).
 * opts may be NULL for all defaults.  The environment variable XAB_POLICY
 * (TIME, STABLE, LEARNED, MEMORY or ACCURACY) overrides the default
 * policy, as the paper's policy file does.  XAB_E_SHAPE for a policy
 * outside the enum. */
int xab_init(xab_ctx **ctx, const xab_init_opts *opts);
void xab_finalize(xab_ctx *ctx);
/* Re-point the context at another stream (hipStream_t). */
int xab_set_stream(xab_ctx *ctx, void *stream);
/* Last error message of this context (static storage owned by ctx). */
const char *xab_last_error(const xab_ctx *ctx);
const char *xab_status_str(int status);

/* ------------------------------------------------------------------ matrix */
/* Wrap a device CRS matrix (section 4.2: the library's only format).
 * rowptr[nrows+1], colind[nnz], val[nnz] of type vt.  Unless
 * XAB_TRUST_INPUT is set, a device pass checks rowptr[0] = 0, monotone
 * rowptr, rowptr[nrows] = nnz, 0 <= col < ncols and, with XAB_SYM_LOWER,
 * square shape and col <= row; failures return XAB_E_STRUCT.  Synchronous. */
int xab_matrix_csr(xab_ctx *ctx, int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *d_rowptr,
                   const int32_t *d_colind, const void *d_val, xab_dtype vt, uint32_t flags,
                   xab_matrix **A);
/* Attach a second copy of the values in the other precision (same
 * structure), e.g. FP32 values for the inner solve of GMRES-IR. */
int xab_matrix_add_values(xab_matrix *A, const void *d_val, xab_dtype vt);
void xab_matrix_destroy(xab_matrix *A);

/* -------------------------------------------------------------------- plan */
/* Build the plan of one implementation with explicit parameters (the
 * setup step that precedes the judge, Table 1): work split arrays,
 * segmented-scan tile descriptors or the symmetric touch map, built by
 * device kernels.  XAB_E_UNSUPPORTED if the variant does not apply. */
int xab_plan_fixed(xab_ctx *ctx, const xab_matrix *A, xab_variant v, const xab_params *p, xab_plan **plan);
void xab_plan_destroy(xab_plan *plan);
/* Read back plan arrays (for checking).  which: 0 nnz-split b / sym tiles b,
 * 1 BSS row_lo, 2 BSS tile_row, 3 BSS carry_row, 4 tm_ptr, 5 tm_tile,
 * 6 tile_ptr, 7 tile_blk, 8 tile_slot, 9 XCB per-block row pointers
 * (8 x (nrows+1), block-major), 10 XCB column indices in block order
 * (the device copy stores each full tile in 16-byte groups interleaved
 * over the lanes; this reports the plain order), bit 31 set on the first
 * entry of each row within its block, 11 SELL
 * row order (original row of each ordered row), 12 SELL ordered row
 * lengths, 13 SELL chunk widths, 14 SELL padded column indices, 15 BCSR
 * block row pointers, 16 BCSR block columns, 17 BCSR position masks, 18
 * SYM_S3 entry-stream walk: column indices with bit 31 set on the first
 * entry of each non-empty row and bit 30 set on an entry that its 64-lane
 * chunk adds after the others (an entry 8, 16, ... positions earlier in
 * the same 512-entry chunk and the same tile has the same column), 19-21
 * SYM_S3 sliced walk: 19 first chunk of each tile (P + 1), 20 chunk
 * widths, 21 padded column-major columns (-1 padding, bit 30 on an entry
 * whose column a lower row of the same chunk has in the same slot).  The
 * arrays of the walk a plan does not take have length 0.
 * *len receives the length; h_out may be NULL to query it.  Synchronous. */
int xab_plan_array(const xab_plan *plan, int32_t which, int32_t *h_out, int64_t *len);
int xab_plan_info(const xab_plan *plan, xab_variant *v, xab_params *p);
/* After the caller has changed the values of the plan's matrix in place
 * (same rowptr and colind, same value arrays), re-read them into the
 * plan's own copies: the column-blocked copy (XCB), the padded copy
 * (SELL), the 4 x 4 blocks (BCSR) and the sliced copy (SYM_S3's sliced
 * walk), keeping the plan's structure (tiles, orders, masks); the other
 * plans read the caller's values directly and need nothing.  The
 * matrix's cached Jacobi diagonal is dropped (the next solve recomputes
 * it).  Waits for the context stream first.  Errors: XAB_E_NULL,
 * XAB_E_NOMEM, XAB_E_DEVICE.  Synchronous. */
int xab_plan_refresh(xab_plan *plan);

/* -------------------------------------------------------------------- SpMV */
/* y = A x for a general matrix.  Value precision = xt (the matrix must hold
 * values of that type).  Supported (x, y, accumulate): (F64, F64, F64),
 * (F32, F32, F32), (F32, F32, F64), (F32, F64, F64).  x has ncols entries,
 * y nrows; they must not overlap.  Asynchronous. */
int xab_spmv_csr(xab_ctx *ctx, const xab_plan *plan, const void *d_x, xab_dtype xt, void *d_y, xab_dtype yt,
                 xab_dtype acc);
/* y = (L + L_strict^T) x for an XAB_SYM_LOWER matrix. Same precisions;
 * XAB_SYM_S3 accumulates in FP64 also when FP32 accumulation is asked for
 * (its tile sums take one LDS atomic add per entry, and the FP32 one runs
 * about 20x slower than the FP64 one on gfx950), so its FP32-accumulation
 * result is its FP64-accumulation result. */
int xab_spmv_sym(xab_ctx *ctx, const xab_plan *plan, const void *d_x, xab_dtype xt, void *d_y, xab_dtype yt,
                 xab_dtype acc);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): y = A x
 * for a general CSR matrix given by its arrays, with no matrix handle, no
 * plan and no device allocation.  It runs the branchless segmented scan
 * (XAB_BSS, 256 * j_per_lane entries per workgroup, j_per_lane a power of
 * two in [1, 32]) and gives the result of xab_spmv_csr with a BSS plan of
 * the same j_per_lane, bit for bit.  Its tile descriptors and carries live
 * in a library-owned device buffer of XAB_NOALLOC_SCRATCH_BYTES on each GPU
 * (set up by xab_init, held until the process ends), which limits the
 * matrix to ceil(nnz / (256 * j_per_lane)) <= XAB_NOALLOC_MAX_TILES tiles
 * (XAB_E_SHAPE beyond).  All calls on one GPU share that buffer: calls
 * that overlap in time on one GPU (other streams or contexts) race, so
 * order them on one stream.  The input is trusted (no validation pass):
 * rowptr[nrows + 1] monotone from 0 to nnz, 0 <= colind < ncols.  Value
 * precision = xt; precisions, alignment and aliasing as for xab_spmv_csr.
 * Asynchronous. */
#define XAB_NOALLOC_SCRATCH_BYTES (8u << 20)
#define XAB_NOALLOC_MAX_TILES 262000
int xab_spmv_csr_noalloc(xab_ctx *ctx, int32_t nrows, int32_t ncols, int64_t nnz, const int32_t *d_rowptr,
                         const int32_t *d_colind, const void *d_val, int32_t j_per_lane, const void *d_x,
                         xab_dtype xt, void *d_y, xab_dtype yt, xab_dtype acc);

/* Average device time of one SpMV with this plan: `warmup` untimed calls,
 * then `reps` calls between two events on the context stream.
 * Synchronous.  Writes milliseconds per call to *ms. */
int xab_time_spmv(xab_ctx *ctx, const xab_plan *plan, const void *d_x, xab_dtype xt, void *d_y, xab_dtype yt,
                  xab_dtype acc, int32_t warmup, int32_t reps, float *ms);

/* ---------------------------------------------------------------- selector */
typedef struct {
    int32_t chosen;                     /* class index */
    float time_ms[XAB_NCLASSES];        /* measured (TIME) or predicted (LEARNED) cost; <0 = invalid class */
    float select_ms;                    /* wall time spent selecting, plan builds included */
    int32_t valid[XAB_NCLASSES];        /* 1 if the class applies to this matrix */
    int64_t bytes[XAB_NCLASSES];        /* device bytes of the class's plan (TIME, MEMORY); -1 = not set up */
} xab_select_info;

/* Choose an implementation under `policy` and return its plan (the
 * run-time judge, section 3.1 before-execution tuning): TIME builds every
 * valid class, times each over 1 warm-up plus 4 runs (minimum taken) and
 * keeps the fastest (lowest class index on ties); STABLE returns the fixed
 * default (NNZ tile_nnz 2048, or SYM_S3 class 11); LEARNED evaluates the
 * cost model on the matrix features; ACCURACY chooses as TIME does;
 * MEMORY sets every valid class up once
 * to learn its plan's bytes, then times, as TIME does, only the classes
 * within 1/64 of the matrix's own bytes (row pointers, columns, values) of
 * the least, and keeps the fastest of them.  Timing runs use FP64 (or the
 * only precision the matrix holds).  info may be NULL.  Synchronous. */
int xab_select(xab_ctx *ctx, const xab_matrix *A, xab_policy policy, xab_plan **plan, xab_select_info *info);

/* The decision rule TIME and MEMORY apply to their measurements (section
 * 3.1: the fastest implementation is kept): over the n classes with
 * valid[k] != 0 and a finite time_ms[k] >= 0, the least time, the lowest
 * index among equal times.  *chosen receives the class, -1 when none
 * qualifies (return XAB_E_UNSUPPORTED).  Host only, no device work; for
 * checking the rule on given tables.  Errors: XAB_E_NULL, XAB_E_SHAPE
 * (n < 0). */
int xab_select_rule(const float *time_ms, const int32_t *valid, int32_t n, int32_t *chosen);
/* 1 if selector class k applies to a matrix with (sym != 0) or without
 * lower symmetric storage, 0 if not, XAB_E_SHAPE for k outside the
 * classes.  Host only. */
int xab_class_applies(int32_t k, int32_t sym);

/* Device memory held by a plan (its own arrays: partitions, descriptors,
 * partials and any re-laid-out copy of the matrix), in bytes; -1 for NULL.
 * The matrix's own arrays are the caller's and not counted. */
int64_t xab_plan_bytes(const xab_plan *plan);

/* The 12 selector features of A (device statistics pass, exact integer
 * arithmetic).  h_out[12]: log2 n, log2 nnz, mean row length, log2(1 +
 * variance of row length), log2 max length, log2(max/mean), bandwidth/n,
 * symmetric flag, empty-row fraction, fraction of rows longer than 64,
 * mean |i-j|/n, fraction of entries in rows longer than 4x the mean.
 * h_stats (may be NULL) receives the 9 int64 statistics behind them.
 * Synchronous. */
int xab_features(xab_ctx *ctx, const xab_matrix *A, float *h_out, int64_t *h_stats);

/* Cost model: MLP 12-64-64-K with K = XAB_NCLASSES, FP32, ReLU, outputs =
 * predicted log2(t_k / t_best).  Parameters in the flat layout W1[64x12]
 * b1[64] W2[64x64] b2[64] W3[Kx64] b3[K] (row-major, out x in), preceded by the
 * feature standardisation mean[12] and std[12].  XAB_MLP_NPARAMS counts
 * only the network. */
#define XAB_MLP_NPARAMS (64 * 12 + 64 + 64 * 64 + 64 + XAB_NCLASSES * 64 + XAB_NCLASSES)
int xab_selector_set(xab_ctx *ctx, const float *h_params, const float *h_mean, const float *h_std);
int xab_selector_get(xab_ctx *ctx, float *h_params, float *h_mean, float *h_std);
int xab_selector_save(xab_ctx *ctx, const char *path);
int xab_selector_load(xab_ctx *ctx, const char *path);

typedef struct {
    int32_t epochs;      /* passes over the training set (300) */
    int32_t batch;       /* mini-batch size (128) */
    float lr;            /* Adam step size (1e-3) */
    float beta1, beta2, eps; /* Adam (0.9, 0.999, 1e-8) */
} xab_train_opts;

typedef struct {
    float final_loss;    /* mean masked MSE of the last epoch */
    float seconds;
} xab_train_info;

/* Train the cost model on the GPU with the library's own forward, backward
 * and Adam kernels.  d_feat[m*12] raw features (standardised internally
 * with the training-set mean/std, which are stored with the weights),
 * d_cost[m*K] measured times (ms; entries with d_valid = 0 ignored),
 * d_valid[m*K] uint8 (K = XAB_NCLASSES).  Starts from the parameters last set with
 * xab_selector_set.  h_order[epochs*m] gives the sample order of each epoch
 * (the caller's shuffle).  h_loss (may be NULL) receives one loss per
 * epoch.  Synchronous. */
int xab_selector_train(xab_ctx *ctx, const float *d_feat, const float *d_cost, const uint8_t *d_valid,
                       int32_t m, const int32_t *h_order, const xab_train_opts *opts, float *h_loss,
                       xab_train_info *info);
/* Raw MLP evaluation on standardised or raw features (for checking):
 * d_feat[m*12] -> d_out[m*12].  raw != 0 applies the stored standardisation
 * first. Asynchronous. */
int xab_selector_forward(xab_ctx *ctx, const float *d_feat, int32_t m, int32_t raw, float *d_out);
/* One loss/gradient evaluation (for checking): d_grad[XAB_MLP_NPARAMS],
 * targets are d_y (already log2 cost ratios), mask d_valid; features are
 * used as given.  Synchronous; *loss receives the loss. */
int xab_selector_loss_grad(xab_ctx *ctx, const float *d_feat, const float *d_y, const uint8_t *d_valid,
                           int32_t m, float *d_grad, float *loss);

/* ------------------------------------------------------------------ Krylov */
typedef enum { XAB_MODE_FP64 = 0, XAB_MODE_IR = 1 } xab_krylov_mode;
typedef enum { XAB_PRECOND_NONE = 0, XAB_PRECOND_JACOBI = 1 } xab_precond;
/* Orthogonalisation of the Arnoldi step (section 3.2.2): DGKS (classical
 * Gram-Schmidt, repeated when the norm fell below 1/sqrt(2) of the
 * incoming one), CGS (once), MGS (column by column), BCGS (blocks of 4
 * columns: CGS inside a block, blocks in order); POLICY is the accuracy
 * policy of section 3.3.2: MGS when the requirement of the orthogonalised
 * solve is <= 1e-10 (tol in FP64 mode, inner_tol in IR mode), else BCGS,
 * and after a fault convergence (a cycle ended on its recurrence residual
 * but the true residual missed tol; FP64 mode) DGKS with a tenfold
 * narrower recurrence threshold. */
typedef enum {
    XAB_ORTHO_DGKS = 0,
    XAB_ORTHO_CGS = 1,
    XAB_ORTHO_MGS = 2,
    XAB_ORTHO_BCGS = 3,
    XAB_ORTHO_POLICY = 4
} xab_ortho;

typedef struct {
    int32_t m;            /* restart length (30) */
    double tol;           /* relative true residual ||b - Ax|| / ||b|| (1e-10) */
    int64_t maxiter;      /* Arnoldi steps / iterations in total */
    double max_time_s;    /* wall-clock limit (<= 0: none) */
    int32_t mode;         /* xab_krylov_mode */
    int32_t precond;      /* xab_precond (right preconditioning) */
    double inner_tol;     /* IR: inner relative residual (1e-6) */
    int32_t graph;        /* batched BiCGStab: capture one iteration in a HIP graph */
    int32_t check_every;  /* batched BiCGStab: iterations between host convergence checks */
    int32_t restart_step; /* GMRES restart-length tuning (0 = fixed m): grow m by this much after a
                             cycle whose residual samples have an MM ratio below mm_ratio */
    int32_t m_max;        /* GMRES restart-length tuning: upper bound on m (<= 63) */
    double mm_ratio;      /* GMRES restart-length tuning: stagnation threshold on the MM ratio */
    int32_t ortho;        /* GMRES: xab_ortho (0 = DGKS) */
} xab_krylov_opts;

typedef struct {
    int64_t iters;        /* Arnoldi steps (GMRES) or iterations (BiCGStab) */
    int64_t restarts;     /* GMRES cycles */
    int64_t refinements;  /* IR outer corrections */
    double true_relres;   /* ||b - A x|| / ||b|| in FP64 at exit */
    double seconds;       /* wall time of the call */
    int32_t status;       /* same as the return value */
    int32_t m_final;      /* GMRES: restart length of the last cycle */
    int32_t faults;       /* GMRES, ortho = POLICY: fault convergences seen */
    int32_t ortho;        /* GMRES: orthogonalisation of the last cycle */
} xab_krylov_info;

/* Restarted GMRES(m) (section 2.2) on A x = b.  d_x holds x0 on entry and
 * the solution on exit (calling again resumes from it).  FP64 mode:
 * everything in FP64.  IR mode: an FP64 outer loop forms r = b - A x with
 * FP64 values and stops when ||r|| / ||b|| <= tol; each correction solves
 * A d = r by GMRES(m) with FP32 values, FP32 basis vectors, FP64 inner
 * products and FP64 Hessenberg/Givens, to inner_tol or one cycle, then
 * x += d in FP64 (needs FP32 values, xab_matrix_add_values).  The plan's
 * variant is used for every SpMV.  Orthogonalisation: classical
 * Gram-Schmidt applied twice (the DGKS scheme, section 3.2.2).
 * Convergence is only declared on the true residual (section 3.3.2).
 * Restart-length tuning (section 3.2.1 with the section 4.3 setting), when
 * restart_step > 0: after every cycle the MM ratio of eq. (1) is taken over
 * that cycle's residual samples (the relative true residual at its start
 * and the relative recurrence residual after each of its steps); below
 * mm_ratio the cycle is judged stagnant and m grows by restart_step, up to
 * m_max.  In IR mode the samples are those of the inner cycle.
 * Inside a cycle the host waits for a step by polling a counter that the
 * step's last kernel writes to pinned host memory; after XAB_STEP_WAIT_MS
 * milliseconds without it (environment variable, default 20; 0 drains at
 * once) it drains the stream instead, with the same result.
 * Synchronous. */
int xab_gmres(xab_ctx *ctx, const xab_plan *plan, const double *d_b, double *d_x, const xab_krylov_opts *opts,
              xab_krylov_info *info);

/* Restarted Lanczos and Arnoldi (section 2.2 solver list, section 4.3
 * setting). */
#define XAB_EIG_LARGEST 0   /* largest algebraic (Arnoldi: largest real part) */
#define XAB_EIG_SMALLEST 1  /* smallest algebraic (Arnoldi: smallest real part) */
#define XAB_EIG_MAGNITUDE 2 /* Arnoldi only: largest magnitude */

typedef struct {
    int32_t nev;        /* wanted eigenpairs, >= 1 */
    int32_t m;          /* basis vectors per cycle, nev < m <= min(63, n) */
    double tol;         /* residual requirement relative to the ||A|| estimate (section 4.3: 1e-8) */
    int64_t maxiter;    /* products with A in the recurrence; <= 0: unlimited */
    double max_time_s;  /* wall-clock limit (the policy's MAXTIME); <= 0: none */
    int32_t which;      /* XAB_EIG_LARGEST or XAB_EIG_SMALLEST */
    int32_t restart_step; /* restart-length tuning: growth of m (0 = off; section 4.3 uses 5) */
    int32_t m_max;      /* tuning: largest m, in [m, min(63, n)] */
    double mm_ratio;    /* tuning: stagnation threshold on the MM ratio of eq. (1) */
    int32_t window;     /* tuning: cycles per MM-ratio sample window (<= 0: 5) */
} xab_eig_opts;

typedef struct {
    int64_t iters;      /* products with A in the recurrence */
    int64_t restarts;   /* thick restarts */
    int32_t nconv;      /* wanted pairs whose residual estimate met tol at exit */
    double anrm;        /* largest |Ritz value| seen: the ||A|| estimate */
    double max_resid;   /* max_i ||A x_i - theta_i x_i|| / anrm over the returned pairs, in FP64 */
    double seconds;     /* wall time of the call */
    int32_t status;     /* same as the return value */
    int32_t m_final;    /* m of the last cycle */
    int32_t nret;       /* eigenvalues returned: nev, or nev + 1 when Arnoldi's nev-th is one of a complex pair */
    int32_t faults;     /* ACCURACY context: convergences the true residuals did not confirm (the threshold
                           was narrowed tenfold after each) */
} xab_eig_info;

/* Thick-restart Lanczos (Wu and Simon's restart; the paper names a
 * restarted Lanczos for symmetric matrices, section 2.2) for the nev
 * eigenpairs of a symmetric A at the chosen end of the spectrum.  The plan
 * may be general (A is then assumed symmetric, not checked) or
 * XAB_SYM_LOWER; every product with A uses the plan's variant in FP64.
 * d_v0 (FP64[n], non-zero) starts the recurrence.  Each new basis vector is
 * orthogonalised against the whole basis (classical Gram-Schmidt with the
 * DGKS second pass); after m vectors the Ritz pairs of T = Q^T A Q are
 * formed, and the solve stops when the residual estimates
 * |beta_m y_{m,i}| of the nev wanted ones are <= tol * anrm; otherwise
 * nev + (m - nev) / 2 Ritz vectors are kept and the recurrence continues.
 * Restart-length tuning (eq. (1) in the manner of section 3.2.1, the
 * section 4.3 growth rule), when restart_step > 0: after every cycle the
 * worst residual estimate of the wanted pairs relative to anrm is sampled;
 * once `window` samples exist since m last changed and their MM ratio is
 * below mm_ratio, m grows by restart_step up to m_max and the samples
 * start afresh.
 * Out: h_evals[nev] (host, wanted end first), d_evecs (device FP64,
 * column-major n x nev, ld = n, orthonormal columns).  XAB_BREAKDOWN when
 * the Krylov space of d_v0 is invariant with dimension below nev;
 * XAB_NOT_CONVERGED / XAB_TIME_LIMIT return the current Ritz pairs.  On a
 * context whose policy is ACCURACY (section 3.3.2) a convergence of the
 * estimates that the true residuals do not confirm (max_resid > tol)
 * narrows the threshold tenfold and the run goes on (at most 8 times,
 * within maxiter and max_time_s); if it cannot be confirmed the call
 * returns XAB_NOT_CONVERGED (info->faults counts the narrowings; the same
 * holds for xab_arnoldi).  Synchronous. */
int xab_lanczos(xab_ctx *ctx, const xab_plan *plan, const double *d_v0, const xab_eig_opts *opts,
                double *h_evals, double *d_evecs, xab_eig_info *info);

/* Implicitly restarted Arnoldi (the paper's restarted Arnoldi for
 * unsymmetric matrices, section 2.2; its restart frequency is what
 * section 4.4.2 tunes) for the nev eigenvalues of a general square A with
 * the largest or smallest real part or the largest magnitude (opts->which).
 * Restart: Sorensen's implicit restart with exact shifts (the m - k
 * unwanted Ritz values as implicit QR shifts, a complex pair as one
 * double-shift step), k = nev + (m - nev) / 2, moved by one so that no
 * complex pair is split.  Recurrence, orthogonalisation, convergence test
 * (residual estimates <= tol * anrm), restart-length tuning and the
 * statuses as for xab_lanczos; nev + 2 <= m <= min(63, n).  When the nev-th
 * wanted value is one of a complex pair its partner is returned too
 * (info->nret = nev + 1).  Out: h_re[nev + 1], h_im[nev + 1] (host, wanted
 * first, a pair as +im then -im); d_evecs (device FP64, column-major
 * n x (nev + 1), ld = n): column i the real eigenvector of a real value, a
 * pair's columns the real and imaginary parts of the eigenvector of its
 * +im member (LAPACK dgeev's layout), each eigenvector of unit norm.
 * info->max_resid = max ||A x - lam x|| / anrm over the returned
 * eigenvectors (complex x for a pair).  Synchronous. */
int xab_arnoldi(xab_ctx *ctx, const xab_plan *plan, const double *d_v0, const xab_eig_opts *opts, double *h_re,
                double *h_im, double *d_evecs, xab_eig_info *info);

/* Batch of independent CSR systems concatenated block-diagonally:
 * system k owns rows [h_row_off[k], h_row_off[k+1]) and entries
 * [h_nnz_off[k], h_nnz_off[k+1]); d_rowptr holds global offsets and
 * d_colind global column indices (inside the system's own row range).
 * The arrays are borrowed and must outlive the batch.  Unless flags has
 * XAB_BATCH_TILES, the batch also keeps its own sliced ELLPACK copy
 * (SELL-C-sigma, C = 64, sigma = 1024: about 12 (FP64) or 8 (FP32) bytes per
 * entry plus padding) and its SpMV runs on that copy; a batch outside the
 * copy's limits (a row longer than 4096 entries, or padding beyond
 * nnz + 64 * longest row), or one whose copy does not fit in device
 * memory, silently uses the segmented-scan tiles instead.
 * Synchronous (validates unless flags has XAB_TRUST_INPUT). */
int xab_batch_csr(xab_ctx *ctx, int32_t nsys, const int64_t *h_row_off, const int64_t *h_nnz_off,
                  const int32_t *d_rowptr, const int32_t *d_colind, const void *d_val, xab_dtype vt,
                  uint32_t flags, xab_batch **batch);
void xab_batch_destroy(xab_batch *batch);
/* Layout the batch's SpMV runs on: 1 = its sliced ELLPACK copy, 0 = the
 * segmented-scan tiles (XAB_BATCH_TILES, or outside the copy's limits);
 * -1 for a null batch. */
int xab_batch_layout(const xab_batch *batch);
/* y = blockdiag(A_k) x over all systems in one persistent launch.
 * Asynchronous. */
int xab_batch_spmv(xab_ctx *ctx, const xab_batch *batch, const void *d_x, void *d_y);
/* BiCGStab (section 2.2, standard van der Vorst form) on every system at
 * once; each system stops when its own recurrence residual meets tol and
 * is masked from then on.  Every system's true residual is recomputed at
 * the end (true_relres).  On a context whose policy is ACCURACY (section
 * 3.3.2) a system whose recurrence met its threshold while the true
 * residual misses tol runs again from its x with the threshold narrowed
 * tenfold (at most 8 times, within maxiter); h_info[k].faults counts the
 * narrowings, and a system whose true residual still misses tol when the
 * narrowings or the iterations run out reports XAB_NOT_CONVERGED.  On other
 * contexts a system's status is its recurrence's outcome: compare
 * true_relres with tol to confirm it.  d_b, d_x in the batch's value
 * precision; d_x holds x0.
 * h_info[nsys] receives per-system results (may be NULL); *all receives
 * the aggregate.  One iteration over all systems is captured as a HIP graph
 * and replayed when opts->graph != 0.  Synchronous. */
int xab_bicgstab(xab_ctx *ctx, const xab_batch *batch, const void *d_b, void *d_x, const xab_krylov_opts *opts,
                 xab_krylov_info *h_info, xab_krylov_info *all);

#ifdef __cplusplus
}
#endif
#endif /* XAB_H */
