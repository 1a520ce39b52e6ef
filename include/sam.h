/*
 * sam.h -- C ABI of the MI355X (gfx950) sparse approximate map library.
 *
 * The library builds the sparse approximate map (SAM) of Islam, Carr and
 * Jacobs, "Optimization of Approximate Maps for Linear Systems Arising in
 * Discretized PDEs": for a source matrix A_k, a target matrix A_0 and a
 * sparsity pattern S it computes
 *
 *     N_k = argmin ||A_k N - A_0||_F  over N with pattern S     (Section 2,
 *                                                              eq. approx_map)
 *
 * column by column as n independent least-squares problems
 * min_m ||A_k(:,J_j) m - A_0(:,j)||_2 with J_j = S(:,j) (end of Section 2),
 * together with the residual R_k = A_k N_k - A_0 (eq. res) and its Frobenius
 * norm, the quality measure of Section 5.  Patterns are the level neighbours
 * of Section 3, S((I + B)^p) with B = S(A~_k), optionally after one of the
 * sparsification rules of Section 4 (global threshold, column threshold tau,
 * fixed count lfil).
 *
 * Conventions shared by every call
 * --------------------------------
 * - All array arguments are DEVICE pointers owned by the caller unless the
 *   comment says "host".  The library never frees caller memory.
 * - Matrices are square n x n in compressed sparse column (CSC) form: colptr
 *   has n+1 int32 entries with colptr[0] = 0 and colptr[n] = nnz, rowind has
 *   nnz int32 row indices strictly ascending inside each column, values are
 *   FP64.  Index counts must fit in int32 (else SAM_ERR_OVERFLOW).
 * - Every call is asynchronous on the given stream (a hipStream_t passed as
 *   sam_stream_t; NULL is the default stream) unless documented as
 *   synchronising.  Host-visible results of asynchronous calls are valid after
 *   the stream has been synchronised.
 * - Numerical failures found inside kernels (a numerically rank-deficient
 *   column block, a non-finite value, an out-of-range index read from caller
 *   data) are recorded in a per-context device status word and reported by
 *   sam_sync_status().  Argument errors are returned immediately.
 * - Device memory is the caller's.  The library allocates none itself except
 *   the 256-byte status block of a context (sam_create).  Every other device
 *   buffer a call needs is passed in: pattern workspaces, plan and sequence
 *   memory, and the scratch of the residual, the row views, the top-k
 *   selection, the penalty scale and the adjoint.  Each is sized by the
 *   matching *_size / *_workspace_size query and must be 256-byte aligned
 *   (any torch allocation is).  The library never frees caller memory.
 *   Memory given to a plan or sequence belongs to it until it is destroyed.
 *   A workspace is free again once the stream has passed the call's kernels.
 * - Concurrency: calls on one context may run on several streams at once if
 *   each uses its own workspace, plan and sequence.  Only the status word is
 *   shared; failures merge into it with an atomic minimum.  Calls that share
 *   a plan must not overlap in time (see sam_build_planned).  The synchronising
 *   calls use the context's status block and its last-error text, so at most
 *   one host thread may call into a context at a time.
 * - Caller structures are checked on the device before any other kernel reads
 *   their indices, in the calls that first receive them: sam_pattern_count,
 *   sam_plan_size / sam_plan_create (A_k, A_0 and S), sam_sequence_size /
 *   sam_sequence_create and sam_apply_prepare.  A bad structure returns
 *   SAM_ERR_UNSORTED with the first bad column in the message.
 * - No call throws; every call returns a sam_status.  sam_last_error() gives a
 *   human-readable message for the last failing call on a context.
 */
#ifndef SAM_MI355X_H
#define SAM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SAM_OK = 0,
    SAM_ERR_ARG = 1,          /* null pointer, negative size, bad enum value  */
    SAM_ERR_SHAPE = 2,        /* inconsistent dimensions between arguments    */
    SAM_ERR_UNSORTED = 3,     /* CSC structure invalid: colptr not monotone,  */
                              /* rows out of range, unsorted or duplicated    */
    SAM_ERR_OVERFLOW = 4,     /* an index count does not fit in int32         */
    SAM_ERR_RANK = 5,         /* a column block is numerically rank deficient */
    SAM_ERR_NONFINITE = 6,    /* NaN or Inf produced                          */
    SAM_ERR_HIP = 7,          /* HIP runtime failure (message has the detail) */
    SAM_ERR_UNSUPPORTED = 8,  /* a column block exceeds the kernels' limits,  */
                              /* or the context has no device                 */
    SAM_ERR_NOMEM = 9         /* device allocation failed                     */
} sam_status;

/* Arithmetic of the least-squares solves.
 * SAM_PREC_F64: Householder QR, solve and residual in FP64; M values FP64.
 * SAM_PREC_F32_REFINE: Householder QR and triangular solves in FP32, then one
 *   seminormal refinement step m += d, d = R^{-1} y, R^T y = A^T (b - A m),
 *   whose residual r = b - A m and A^T r are accumulated in FP64 from the
 *   FP64 inputs; the per-column residual is ||r||^2 - ||y||^2 (+ the A_0
 *   entries outside I_j), the FP64 residual of the unrefined m less the
 *   step's decrease (exact up to rounding in the FP32 factor R); M values
 *   stored FP32. */
typedef enum { SAM_PREC_F64 = 0, SAM_PREC_F32_REFINE = 1 } sam_precision;
/* Calls take the precision as an int32_t holding one of these values (any
 * other value is SAM_ERR_ARG). */

/* Sparsification of A_k before the level expansion (Section 4).  The
 * diagonal is always kept, also when it is not stored. */
typedef enum {
    SAM_SPARSIFY_NONE = 0,    /* B = stored entries of A_k                     */
    SAM_SPARSIFY_GLOBAL = 1,  /* keep |a_ij| * s_ij > thresh, s_ij =           */
                              /* (D_ii D_jj)^(-1/2) (global_scale = -1) or     */
                              /* (D_ii D_jj)^(+1/2) (global_scale = +1, the    */
                              /* printed form); D_ii = |a_ii|, or 1 if zero    */
    SAM_SPARSIFY_COLUMN = 2,  /* keep |a_ij| > (1 - tau) max_i |a_ij|          */
    SAM_SPARSIFY_LFIL = 3     /* keep the diagonal and the lfil-1 largest      */
                              /* off-diagonal magnitudes (ties: smaller row)   */
} sam_sparsify;

typedef void* sam_stream_t;   /* a hipStream_t */

typedef struct {
    int32_t n;                /* order of the matrix                          */
    int32_t nnz;              /* stored entries                               */
    const int32_t* colptr;    /* device, n+1                                  */
    const int32_t* rowind;    /* device, nnz, ascending within each column    */
    const double* val;        /* device, nnz (may be NULL where documented)   */
} sam_csc;

typedef struct {
    int32_t kind;             /* sam_sparsify                                 */
    int32_t power;            /* p >= 1: S = S((I + B)^p)  (Section 3 levels) */
    double thresh;            /* SAM_SPARSIFY_GLOBAL                          */
    int32_t global_scale;     /* -1 (default) or +1, see above                */
    double tau;               /* SAM_SPARSIFY_COLUMN, 0 <= tau <= 1           */
    int32_t lfil;             /* SAM_SPARSIFY_LFIL, >= 1                      */
} sam_pattern_spec;

typedef struct sam_ctx sam_ctx;
typedef struct sam_plan sam_plan;
typedef struct sam_seq sam_seq;

#define SAM_NO_DEVICE (-1)

/* ---------------------------------------------------------------- context */

/* Create a context bound to HIP device `device`: allocates its 256-byte
 * device status block (the status word of the kernels' failures and the flags
 * of the structure checks).  device = SAM_NO_DEVICE gives a host-only
 * context on which every call validates its arguments and then returns
 * SAM_ERR_UNSUPPORTED instead of touching a GPU.
 * Errors: SAM_ERR_ARG (ctx NULL), SAM_ERR_HIP (device not usable),
 * SAM_ERR_NOMEM. */
sam_status sam_create(sam_ctx** ctx, int device);

/* Release the context and its status block (synchronises the device first).
 * ctx may be NULL. */
sam_status sam_destroy(sam_ctx* ctx);

/* Message of the last failing call on ctx (static storage owned by ctx;
 * "" when none).  Valid until the next call on ctx. */
const char* sam_last_error(const sam_ctx* ctx);

/* Name of a status code (static string). */
const char* sam_status_string(sam_status s);

/* Library version string "major.minor.patch" (static). */
const char* sam_version(void);

/* Synchronise `stream`, read and clear the context's device status word.
 * Returns the status of the earliest failing column since the last call
 * (SAM_OK if none) and writes that column to *first_bad_col (host; -1 when
 * none).  Synchronising. */
sam_status sam_sync_status(sam_ctx* ctx, sam_stream_t stream, int32_t* first_bad_col);

/* Check the CSC structure of A on the device: colptr[0] = 0, monotone,
 * colptr[n] = nnz, rows in [0, n), strictly ascending within each column.
 * Synchronising.  Errors: SAM_ERR_UNSORTED with the first bad column in the
 * message. */
sam_status sam_check_csc(sam_ctx* ctx, const sam_csc* A, sam_stream_t stream);

/* ---------------------------------------------------------------- pattern */

/* Bytes of the workspace sam_pattern_count / sam_pattern_fill need for this
 * A_k structure and spec->power (host output).  B = S(A~_k) needs
 * nnz(A_k) + n entries.  An intermediate level of power q (p >= 3) needs at
 * most n min(n, (1 + longest column)^q) entries.  Synchronising: reads
 * colptr to the host and checks it.  Errors: as sam_pattern_count, and
 * SAM_ERR_UNSORTED for a bad colptr. */
sam_status sam_pattern_workspace_size(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec,
                                      size_t* bytes, sam_stream_t stream);

/* Sections 3-4: S = S((I + B)^p), B = S(A~_k) plus the diagonal, with A~_k
 * given by spec->kind.  Column j of S is the set of vertices with a path of
 * length <= p to j in G(B), rows ascending.  First checks A_k's structure.
 * Then counts the pattern in the workspace `ws` (ws_bytes >=
 * sam_pattern_workspace_size): B and the intermediate levels are stored
 * there, the last level is counted.  Returns nnz(S) in *nnz_S (host).
 * Synchronising (the count sizes S on the host).  A_k values are read only
 * for the value-dependent rules.  Errors: SAM_ERR_ARG (power < 1, tau
 * outside [0,1], lfil < 1, bad kind, workspace too small or unaligned),
 * SAM_ERR_UNSORTED (bad structure), SAM_ERR_OVERFLOW (nnz(S) >= 2^31). */
sam_status sam_pattern_count(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, void* ws,
                             size_t ws_bytes, int64_t* nnz_S, sam_stream_t stream);

/* Write the pattern counted by the last sam_pattern_count on ctx into caller
 * arrays S_colptr (n+1) and S_rowind (nnz_S).  Ak, spec and ws must be the
 * ones passed to that count, with ws unchanged since; otherwise SAM_ERR_ARG.
 * Asynchronous. */
sam_status sam_pattern_fill(sam_ctx* ctx, const sam_csc* Ak, const sam_pattern_spec* spec, void* ws,
                            size_t ws_bytes, int32_t* S_colptr, int32_t* S_rowind, sam_stream_t stream);

/* ------------------------------------------------------------------ build */

/* Bytes of plan memory for sam_plan_create on these structures (host
 * output).  The size depends on the gathered entries
 * E = sum_j sum_{l in J_j} nnz(A_k(:,l)), one position byte each, which a
 * kernel counts.  Checks A_k and S first.  Synchronising.  Errors as
 * sam_plan_create. */
sam_status sam_plan_size(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0,
                         const int32_t* S_colptr, const int32_t* S_rowind, int64_t nnz_S, size_t* bytes,
                         sam_stream_t stream);

/* Symbolic analysis of the column problems for the structure of A_k (values
 * ignored), the structure of A_0 (values ignored) and the pattern S:
 * row sets I_j = rows(A_k(:,J_j)) (Section 2: the submatrix of A_k selected
 * by S; rows outside I_j are zero), the position of every A_k and A_0 entry
 * inside its column block, and the size classes (buckets) the numeric kernels
 * run in.  The three structures are checked on the device first.  The plan's
 * arrays are carved from the caller's `mem` (mem_bytes >= sam_plan_size),
 * which the plan owns until sam_plan_destroy.  The plan also keeps pointers
 * to the caller's structure arrays, which must stay valid and unchanged while
 * the plan is used.  Synchronising.
 * Errors: SAM_ERR_SHAPE (n mismatch, S size), SAM_ERR_UNSORTED (a bad
 * structure), SAM_ERR_UNSUPPORTED (a column block larger than the largest
 * kernel class: |I_j| > 128 or |J_j| > 32), SAM_ERR_OVERFLOW, SAM_ERR_ARG
 * (memory too small or unaligned). */
sam_status sam_plan_create(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0,
                           const int32_t* S_colptr, const int32_t* S_rowind, int64_t nnz_S,
                           void* mem, size_t mem_bytes, sam_plan** plan, sam_stream_t stream);

/* Release a plan (NULL allowed).  Synchronises the device first, so work
 * still enqueued on the plan finishes; its memory then returns to the
 * caller. */
sam_status sam_plan_destroy(sam_plan* plan);

/* Shape statistics of a plan (host outputs, any may be NULL): number of
 * columns, max |I_j|, max |J_j|, total gathered entries sum_j nnz(A_k(:,J_j)),
 * and the column count of each of up to 16 buckets (bucket_cols[16]). */
sam_status sam_plan_info(const sam_plan* plan, int32_t* n, int32_t* max_rows, int32_t* max_cols,
                         int64_t* gathered, int32_t* nbuckets, int32_t* bucket_cols);

/* Algorithmic cost of one sam_build_planned on this plan (host outputs, any
 * may be NULL): flops of the dense column blocks, split into FP32 work
 * (Householder QR 2 r c^2 - 2/3 c^3, Q^T b, triangular solves) and FP64 work
 * (refinement residuals; everything for SAM_PREC_F64), with r = |I_j|,
 * c = |J_j| summed over columns; and compulsory HBM bytes
 * 12 nnz(A_k) + 12 nnz(A_0) + 4 nnz(S) + 12 (n+1) + v nnz(S) + 8 n, with
 * v = 4 (FP32 map) or 8 (FP64 map). */
sam_status sam_plan_cost(const sam_plan* plan, int32_t prec, double* flops32, double* flops64,
                         double* bytes);

/* Algorithmic cost of one sam_build_weighted (backward = 0) or one
 * sam_backward (backward = 1) on this plan (host outputs, may be NULL):
 * flops of the stacked (|I_j| + |J_j|) x |J_j| Householder QR, Q^T b and the
 * solves (FP32 in SAM_PREC_F32_REFINE), and of the FP64 refinement pass
 * (one step: r = b - A m, ||r||^2, A^T r, P m).  The adjoint adds the two
 * normal-equation solves of lambda, its residual passes and five flops per
 * gathered entry for the A_k contributions. */
sam_status sam_plan_cost_weighted(const sam_plan* plan, int32_t prec, int32_t backward, double* flops32,
                                  double* flops64);

/* The numeric kernel variants compiled for `prec` (weighted = 0: plain maps,
 * 1: soft-weighted), in their default order.  Each serves column blocks of
 * at most G*R rows (G*R - |J_j| penalty rows aside when weighted) and NC
 * columns; G lanes of a wave64 own one column problem, TC columns are staged
 * per LDS pass.  Host outputs of `capacity` entries (any may be NULL);
 * *count receives the number of variants.  Needs no context and no device. */
sam_status sam_menu(int32_t prec, int32_t weighted, int32_t capacity, int32_t* count, int32_t* G,
                    int32_t* R, int32_t* NC, int32_t* TC);

/* Choose the variants of the plan's plain builds in precision `prec`:
 * `order` lists 1..16 indices into sam_menu(prec, 0); every column is served
 * by the first listed variant its block fits (this is how the size buckets
 * are formed).  Re-sorts the plan's buckets; synchronising.  Errors:
 * SAM_ERR_ARG (bad index or count), SAM_ERR_UNSUPPORTED (some column fits no
 * listed variant; the previous choice stays). */
sam_status sam_plan_select(sam_plan* plan, int32_t prec, const int32_t* order, int32_t count,
                           sam_stream_t stream);

/* Numeric SAM build on a plan (Section 2): for every column j solve
 * min ||A_k(I_j,J_j) m - A_0(I_j,j)||_2 by Householder QR and back
 * substitution (prec selects FP64 or FP32 + FP64-residual refinement), write
 * m into M_val[S_colptr[j] .. S_colptr[j+1]) (double for SAM_PREC_F64, float
 * for SAM_PREC_F32_REFINE), and the squared column residual
 * rho_j = ||A_k(:,J_j) m - A_0(:,j)||^2 into col_res2[j] (optional, may be
 * NULL).  res2 (optional device scalar) receives sum_j rho_j =
 * ||A_k M - A_0||_F^2, summed in a fixed order (bitwise reproducible).
 * Ak_val and A0_val are the values matching the plan's structures.
 * Uses only the plan's memory; safe to capture in a HIP graph.  Calls on
 * one plan (builds and sam_backward) must not overlap in time: they share
 * the plan's scratch (column residuals when col_res2 is NULL, the residual
 * sum's partials).
 * Async errors (sam_sync_status): SAM_ERR_RANK, SAM_ERR_NONFINITE. */
sam_status sam_build_planned(sam_plan* plan, const double* Ak_val, const double* A0_val,
                             int32_t prec, void* M_val, double* col_res2, double* res2,
                             sam_stream_t stream);

/* Bytes of the workspace sam_build needs (host output): the plan of the
 * column problems (sam_plan_size; the same for both precisions).
 * Synchronising. */
sam_status sam_workspace_size(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0,
                              const int32_t* S_colptr, const int32_t* S_rowind, int64_t nnz_S,
                              int32_t prec, size_t* bytes, sam_stream_t stream);

/* One-shot build (Section 2): sam_plan_create in `ws` (ws_bytes >=
 * sam_workspace_size), then sam_build_planned.  The planning is synchronising
 * (host-side sizing); the numeric launches are left on the stream and read
 * ws until it reaches them.  Outputs and errors as sam_plan_create and
 * sam_build_planned. */
sam_status sam_build(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0,
                     const int32_t* S_colptr, const int32_t* S_rowind, int64_t nnz_S,
                     int32_t prec, void* M_val, double* col_res2, double* res2,
                     void* ws, size_t ws_bytes, sam_stream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): sam_build
 * with the plan of the column problems in a fixed 48 MiB device array of the
 * library instead of a caller workspace.  Each GPU the library runs on holds
 * one such array until the process ends.  Problems whose plan needs more
 * (sam_workspace_size > 48 MiB; the 512 x 512 level-2 map needs about
 * 31 MiB) are refused with SAM_ERR_UNSUPPORTED before any kernel runs.
 * Arguments, outputs and the synchronising planning are those of sam_build;
 * the numeric launches read the array until the stream reaches them.  Every
 * call on a GPU shares that GPU's array, which keeps the last call's
 * contents: calls on one stream are ordered, but calls that overlap on one
 * GPU (other streams, threads or contexts) race on it.  Not capturable (the
 * planning synchronises).  Allocates nothing. */
sam_status sam_build_noalloc(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0,
                             const int32_t* S_colptr, const int32_t* S_rowind, int64_t nnz_S,
                             int32_t prec, void* M_val, double* col_res2, double* res2,
                             sam_stream_t stream);

/* --------------------------------------------------------------- residual */

/* Bytes of the workspace of sam_residual for order n and nnz(A_0) (host
 * output; n doubles of column residuals and a reduction temporary). */
sam_status sam_residual_workspace_size(int32_t n, int32_t nnz_A0, size_t* bytes);

/* Section 2 eq. (res): res2 = ||A_k M - A_0||_F^2 recomputed explicitly from
 * the stored map M (pattern M_colptr/M_rowind, values M_val in double for
 * SAM_PREC_F64 or float for SAM_PREC_F32_REFINE), independently of the
 * build's per-column residuals; a02 (optional) = ||A_0||_F^2, so that the
 * relative residual of Section 5 is sqrt(res2 / a02).  Both are device
 * scalars, summed in a fixed order.  ws: sam_residual_workspace_size bytes.
 * Asynchronous.  A_k and A_0 are taken as valid (sam_check_csc); a row of M
 * outside [0, n) is reported through the status word. */
sam_status sam_residual(sam_ctx* ctx, const sam_csc* Ak, const sam_csc* A0,
                        const int32_t* M_colptr, const int32_t* M_rowind, int64_t nnz_M,
                        const void* M_val, int32_t prec, double* res2, double* a02,
                        void* ws, size_t ws_bytes, sam_stream_t stream);

/* ------------------------------------------------------------------ apply */

/* Bytes of the workspace of sam_apply_prepare for order n (host output). */
sam_status sam_apply_workspace_size(int32_t n, size_t* bytes);

/* Row view of a CSC pattern for y = M x: T_rowptr (n+1), T_colind (nnz) and
 * T_perm (nnz) such that row i of M is {(T_colind[e], M_val[T_perm[e]])} for
 * e in [T_rowptr[i], T_rowptr[i+1]), columns ascending.  Checks the pattern
 * first (synchronising); the view is built asynchronously in the caller's
 * arrays with ws (sam_apply_workspace_size bytes) as scratch. */
sam_status sam_apply_prepare(sam_ctx* ctx, int32_t n, const int32_t* M_colptr,
                             const int32_t* M_rowind, int64_t nnz, int32_t* T_rowptr,
                             int32_t* T_colind, int32_t* T_perm, void* ws, size_t ws_bytes,
                             sam_stream_t stream);

/* T_val[e] = M_val[T_perm[e]] for e in [0, nnz): M's values in the row
 * view's order, so that sam_apply with T_perm = NULL reads them as contiguous
 * runs (one pass per map, before the Krylov iterations that apply it).
 * M_val and T_val (nnz values, caller-owned) are double or float per prec.
 * Asynchronous; allocates nothing. */
sam_status sam_apply_permute(sam_ctx* ctx, int64_t nnz, const int32_t* T_perm,
                             const void* M_val, int32_t prec, void* T_val, sam_stream_t stream);

/* y = M x (the map applied inside a Krylov iteration; Section 1: the map
 * updates a preconditioner), FP64 accumulation: four lanes per row, each
 * summing every fourth entry of the row in ascending order, then the four
 * partials in a fixed order (bitwise reproducible from call to call).  M_val
 * is double or float per prec; T_perm = NULL means M_val is already in the
 * row view's order (sam_apply_permute).  Allocates nothing. */
sam_status sam_apply(sam_ctx* ctx, int32_t n, const int32_t* T_rowptr, const int32_t* T_colind,
                     const int32_t* T_perm, const void* M_val, int32_t prec,
                     const double* x, double* y, sam_stream_t stream);

/* --------------------------------------------------------------- sequence */

/* Bytes of sequence memory for sam_sequence_create with the same arguments
 * (host output).  ws is a pattern workspace for Ak_struct and spec
 * (sam_pattern_workspace_size).  In it the structural pattern
 * S((I + S(A_k))^p) is counted, the bound of every source's pattern.  Checks
 * both structures.  Synchronising.  Errors as sam_sequence_create. */
sam_status sam_sequence_size(sam_ctx* ctx, const sam_csc* A0, const sam_csc* Ak_struct,
                             const sam_pattern_spec* spec, int32_t n_src, int32_t prec,
                             int32_t replan_each_run, void* ws, size_t ws_bytes, size_t* bytes,
                             sam_stream_t stream);

/* A sequence A_1..A_N mapped to the target A_0 (Section 2: every source is
 * mapped back to A_0).  All sources share the structure of `Ak_struct`
 * (values ignored); their values are passed per run.  The pattern follows
 * `spec` per source: when the rule does not depend on values
 * (SAM_SPARSIFY_NONE) the pattern and plan are computed once here, unless
 * `replan_each_run` is nonzero; value-dependent rules are recomputed for every
 * source inside each run, sized to the unsparsified bound.  Everything lives
 * in the caller's `mem` (mem_bytes >= sam_sequence_size), owned by the
 * sequence until sam_sequence_destroy.  The first run with a given set of
 * pointers is captured into a HIP graph; later runs with the same pointers
 * replay it.  M_vals[k] must hold nnz_bound entries (sam_sequence_info).
 * Errors: SAM_ERR_ARG also for n = 0 (nothing to map) and for memory too
 * small; SAM_ERR_UNSORTED (a bad structure).  Synchronising. */
sam_status sam_sequence_create(sam_ctx* ctx, const sam_csc* A0, const sam_csc* Ak_struct,
                               const sam_pattern_spec* spec, int32_t n_src, int32_t prec,
                               int32_t replan_each_run, void* mem, size_t mem_bytes, sam_seq** seq,
                               sam_stream_t stream);

sam_status sam_sequence_destroy(sam_seq* seq);

/* nnz bound per map (host): the size M_vals[k] must have. */
sam_status sam_sequence_info(const sam_seq* seq, int64_t* nnz_bound);

/* Copy the pattern of source k as computed by the last run (static mode:
 * the shared pattern) into caller arrays S_colptr (n+1) and S_rowind (at most
 * nnz_bound entries); *nnz_S (host) receives its size.  Synchronising. */
sam_status sam_sequence_pattern(sam_seq* seq, int32_t k, int32_t* S_colptr, int32_t* S_rowind, int64_t* nnz_S,
                                sam_stream_t stream);

/* sam_plan_select for the sequence's precision; the next run re-captures. */
sam_status sam_sequence_select(sam_seq* seq, const int32_t* order, int32_t count, sam_stream_t stream);

/* Build every map of the sequence: Ak_vals (host array of n_src device
 * pointers), M_vals (host array of n_src device pointers), res2 (device,
 * n_src doubles: ||A_k M_k - A_0||_F^2).  Graph-replayed after the first call
 * with the same pointers.  Allocates nothing after the first call. */
sam_status sam_sequence_run(sam_seq* seq, const double* const* Ak_vals, void* const* M_vals,
                            double* res2, sam_stream_t stream);

/* -------------------------------------------------------- weights, adjoint */

/* Soft-weighted map (not in the paper; a differentiable relaxation of the
 * pattern choice): column j solves
 *     min ||A_k(I_j,J_j) m - A_0(I_j,j)||^2 + sum_l p_l m_l^2,
 *     p_l = mu (1/w_l - 1),  w in (0, 1] aligned with S's entries,
 * as the stacked least-squares problem [A; diag(sqrt p)] (w = 1 leaves an
 * entry unpenalised, w -> 0 removes it).  col_res2 / res2 exclude the
 * penalty.  Only SAM_PREC_F32_REFINE (with one refinement step) and
 * SAM_PREC_F64 are accepted.  Allocates nothing. */
sam_status sam_build_weighted(sam_plan* plan, const double* Ak_val, const double* A0_val,
                              const double* w, double mu, int32_t prec, void* M_val,
                              double* col_res2, double* res2, sam_stream_t stream);

/* Bytes of the workspace of sam_backward on this plan (host output): a
 * staging double per gathered entry, an offset per S entry, the row view of
 * S and its temporaries. */
sam_status sam_backward_workspace_size(const sam_plan* plan, size_t* bytes);

/* Build the row view of S (which columns j contain row l, ascending j) in
 * ws for sam_backward on this plan.  Asynchronous. */
sam_status sam_backward_prepare(sam_plan* plan, void* ws, size_t ws_bytes, sam_stream_t stream);

/* Adjoint of L = dL * ||A_k M - A_0||_F^2 for the soft-weighted map M: the
 * QR of each stacked block is recomputed (nothing is stored by the forward
 * pass), lambda = (A^T A + P)^{-1} 2 A^T r with r = A m - b (FP32 mode: two
 * FP64-residual refinement steps on lambda), and
 *   gAk  (nnz(A_k), overwritten): sum over columns j of
 *        dL (2 r m^T - r lambda^T - (A lambda) m^T) at the stored entries,
 *   gA0  (nnz(A_0), overwritten): dL (-2 r + A lambda) on I_j, dL 2 a_0(i,j)
 *        outside I_j,
 *   gw   (nnz_S, optional):       dL mu lambda_l m_l / w_l^2,
 *   loss (optional device scalar): ||A_k M - A_0||_F^2 (not scaled by dL).
 * The A_k gradient is summed per entry over the columns in ascending order
 * from the staging part of ws (no atomics: bitwise reproducible).  ws must
 * have been prepared for this plan by sam_backward_prepare and not changed
 * since (else SAM_ERR_ARG); its staging part is rewritten by every call.
 * Asynchronous; calls on one plan must not overlap in time. */
sam_status sam_backward(sam_plan* plan, const double* Ak_val, const double* A0_val,
                        const double* w, double mu, double dL, int32_t prec,
                        double* gAk, double* gA0, double* gw, double* loss,
                        void* ws, size_t ws_bytes, sam_stream_t stream);

/* ------------------------------------------------------ adaptive patterns */

/* The paper leaves adaptive patterns as future work (end of Section 2;
 * Section 6).  These calls build one from the soft-weighted map's adjoint:
 * weight the entries of a candidate pattern S (e.g. S(A_k^2)) that are not in
 * a base pattern B (e.g. S(A_k)), take dL/dw from sam_backward, and keep per
 * column the base entries plus the k candidates whose admission lowers the
 * loss fastest. */

/* w[e] (device, nnz_S entries, overwritten) = w_base where entry e of S is
 * also in B (same column and row), w_cand elsewhere.  S and B are CSC
 * patterns on the device with rows ascending per column.  Errors:
 * SAM_ERR_ARG (NULL, negative sizes), SAM_ERR_SHAPE / SAM_ERR_UNSORTED (the
 * column pointers, checked on the host), SAM_ERR_OVERFLOW.  Synchronising
 * (the column-pointer check). */
sam_status sam_candidate_weights(sam_ctx* ctx, int32_t n, const int32_t* S_colptr, const int32_t* S_rowind,
                                 int64_t nnz_S, const int32_t* B_colptr, const int32_t* B_rowind, int64_t nnz_B,
                                 double w_base, double w_cand, double* w, sam_stream_t stream);

/* Bytes of the workspace of sam_pattern_topk for order n (host output). */
sam_status sam_topk_workspace_size(int32_t n, size_t* bytes);

/* Top-k selection: column j of the output keeps, in S's (ascending) order,
 * every entry of S(:, j) with w >= 1 and the k entries with w < 1 that have
 * the smallest grad (NaN counts as +inf; ties go to the smaller row).  grad
 * is typically sam_backward's gw (negative: admitting the entry lowers the
 * loss).  out_colptr (n+1) and out_rowind (at most nnz_S entries) are device
 * arrays of the caller; *nnz_out (host) receives the output size.  ws:
 * sam_topk_workspace_size bytes.  Errors as for sam_candidate_weights, and
 * SAM_ERR_ARG for k < 0.  Synchronising. */
sam_status sam_pattern_topk(sam_ctx* ctx, int32_t n, const int32_t* S_colptr, const int32_t* S_rowind,
                            int64_t nnz_S, const double* w, const double* grad, int32_t k, int32_t* out_colptr,
                            int32_t* out_rowind, int64_t* nnz_out, void* ws, size_t ws_bytes,
                            sam_stream_t stream);

/* Bytes of the workspace of sam_penalty_scale for nnz(A_k) (host output). */
sam_status sam_penalty_workspace_size(int32_t nnz, size_t* bytes);

/* The penalty scale of the soft weights: *mu (host) = ||A_k||_F^2 / n, the
 * mean squared column norm (a fixed scalar, not differentiated).  ws:
 * sam_penalty_workspace_size bytes.  Errors: SAM_ERR_ARG (NULL, n = 0, no
 * values).  Synchronising. */
sam_status sam_penalty_scale(sam_ctx* ctx, const sam_csc* Ak, double* mu, void* ws, size_t ws_bytes,
                             sam_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* SAM_MI355X_H */
