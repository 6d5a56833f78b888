/*
 * miqr: MI355X-native Householder QR and least squares (C ABI).
 *
 * Method: "A 3D Parallel Algorithm for QR Decomposition" (Ballard, Demmel,
 * Grigori, Jacquelin, Knight).  The factorisation is the Elmroth-Gustavson
 * recursion QR-EG (Alg. 2): split the columns in two, factor the left half,
 * update the right half with the compact-WY product C <- C - V (T^T (V^T C))
 * (Sec. 2.3, eq. for the basis-kernel update), factor the lower right block,
 * and assemble V and T (Sec. 2.3, basis-kernel assembly).  Below a column
 * cutoff the base case is the TSQR panel factorisation of 1D-CAQR-EG (Sec. 5,
 * Sec. 6.1, App. C): local QR of row blocks, a reduction tree over the stacked
 * R factors, a downsweep that forms the leading columns of Q, and Householder
 * reconstruction (App. C.2) of V, T and R.
 *
 * Conventions shared by every entry point
 *  - Matrices are column-major: element (i, j) of a matrix with leading
 *    dimension ld is at p[i + j*ld].  Sizes and leading dimensions are int64_t.
 *  - Matrix pointers are DEVICE pointers (HIP device memory of the handle's
 *    device) unless a parameter says "host".  The caller owns every matrix it
 *    passes; the library never frees or retains them past the call.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Every call is enqueued on that stream and returns without waiting,
 *    unless a host-side output (qr_info) is requested, in which case the call
 *    synchronises the stream before returning.
 *  - Arguments are validated before anything is enqueued; on MIQR_EINVAL no
 *    device memory is touched.
 *  - A handle is not thread-safe; use one handle per host thread.  Calls on one
 *    handle that overlap on different streams race on its workspace.
 *
 * Output representation (Sec. 2.3, "Householder representation"): after
 * qr_factor, A's upper triangle holds R (n x n), its strict lower trapezoid
 * holds V (unit lower trapezoidal, unit diagonal implicit), and T (n x n upper
 * triangular) satisfies Q = I - V T V^T, A = Q R.  Reflector signs follow
 * R_jj = -sign(alpha_j) * ||x_j|| (the sign that Householder reconstruction
 * selects with S_jj = sgn(X_jj)), so the result matches unblocked Householder
 * QR with the LAPACK dlarfg rule.
 */
#ifndef MIQR_H
#define MIQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum miqr_status {
    MIQR_OK = 0,
    MIQR_EINVAL = 1,    /* invalid argument; nothing was enqueued */
    MIQR_ENOMEM = 2,    /* workspace allocation failed */
    MIQR_EHIP = 3,      /* a HIP runtime or launch error */
    MIQR_ESINGULAR = 4, /* lstsq: R has an exactly zero diagonal entry */
    MIQR_ENOCONV = 5,   /* refinement did not reach its target; FP64 fallback used */
    MIQR_EBUSY = 6,     /* server back-pressure: no slot or memory right now */
    MIQR_ENOTSUP = 7    /* option combination not supported */
} miqr_status;

typedef enum miqr_precision {
    MIQR_FP64 = 0,       /* every step in FP64 (FP64 MFMA for the updates) */
    MIQR_MIXED_FP32 = 1, /* trailing-update GEMMs on FP32 MFMA, FP32 accumulate */
    MIQR_MIXED_BF16 = 2  /* trailing-update GEMMs on BF16 MFMA, FP32 accumulate */
} miqr_precision;

/* Layout of the kernel T returned by qr_factor. */
typedef enum miqr_t_layout {
    /* n x n upper triangular T of Alg. 2's assembly: Q = I - V T V^T. */
    MIQR_T_FULL = 0,
    /* The T-avoiding variant of Sec. 8.4: the top level of the recursion is a
     * right-looking loop over panels of nb columns, each factored by Alg. 2,
     * and only each panel's own T is formed.  T is nb x n: panel k (columns
     * k nb .. k nb + w_k - 1, w_k = min(nb, n - k nb)) keeps its w_k x w_k
     * upper triangular T_k in rows 0 .. w_k - 1 of its columns, zeros below;
     * Q = Q_0 Q_1 ... Q_{K-1} with Q_k = I - V_k T_k V_k^T (V_k: panel k's
     * columns of V).  nb = n gives FULL. */
    MIQR_T_BLOCKED = 1
} miqr_t_layout;

typedef struct miqr_ctx *miqr_handle;

/* Tuning and output options.  A NULL qr_opts* means all defaults.  Zero in a
 * tuning field means "choose automatically": the library's cost model (the
 * alpha-beta-gamma model of Sec. 3 with launches for messages, fitted on
 * MI355X) picks the value, per shape; qr_plan reports the choice. */
typedef struct qr_opts {
    int64_t b;         /* Alg. 2 threshold: nodes at most b columns wide are
                          base cases (1D-CAQR-EG of width <= b, whose own base
                          case is a TSQR panel of width <= bstar).  0 .. 4096 */
    int64_t leaf_rows; /* TSQR leaf row-block height: 128 or 256 */
    int64_t chain;     /* leaf blocks reduced in sequence by one workgroup */
    int64_t arity;     /* TSQR tree arity above the leaf chains (>= 2) */
    int32_t precision; /* miqr_precision */
    int32_t normalize; /* nonzero: store R~ = D R with D = diag(sign(R_jj)) so
                          that diag(R~) >= 0; then A = Q D R~ with
                          Q = I - V T V^T.  sign_out must be given. */
    double *sign_out;  /* device, n doubles: D (+1/-1), written when normalize */
    double *Q;         /* device, optional m x n explicit thin Q (Q D when
                          normalize) */
    int64_t ldq;
    int64_t bstar;     /* base-case panel width b* (TSQR panels), 1 .. 64,
                          at most b; 0: automatic (b when b <= 64) */
    int64_t nb;        /* MIQR_T_BLOCKED: width of the top-level panels,
                          0 .. 4096 (0: automatic) */
    int32_t t_layout;  /* miqr_t_layout (0: MIQR_T_FULL) */
    int32_t no_lookahead; /* MIQR_T_BLOCKED: nonzero keeps every step on the
                          caller's stream; otherwise panel k + 1 is factored
                          while an internal stream applies panel k to the
                          columns beyond it */
} qr_opts;

/* Host-side result of qr_lstsq. */
typedef struct qr_info {
    int32_t iterations;     /* refinement iterations performed (0 for FP64) */
    int32_t fallback;       /* 1 if the mixed form fell back to FP64 */
    int32_t precision_used; /* miqr_precision of the factors finally used */
    int32_t singular_index; /* 1-based index j with R_jj == 0, or 0 */
    double backward_error;  /* max over right-hand sides of
                               ||A^T r|| / (||A||_F (||A||_F ||x|| + ||r||)) */
} qr_info;

/* Create a handle bound to HIP device `device`; it owns a lazily grown device
 * workspace.  Returns MIQR_EINVAL for a bad device index. */
miqr_status miqr_create(miqr_handle *handle, int device);

/* Release the handle and its workspace.  Pending work on streams that use the
 * handle must have completed. */
miqr_status miqr_destroy(miqr_handle handle);

/* Static description of a status code. */
const char *miqr_status_string(miqr_status status);

/* Text of the last error recorded on the handle (empty if none). */
const char *miqr_last_error(miqr_handle handle);

/* Bytes of device workspace qr_factor needs for this shape (informational;
 * the handle allocates it on first use).  0 for invalid sizes or options.
 * Host only. */
int64_t qr_workspace_size(int64_t m, int64_t n, const qr_opts *opts);

/* Rows of T that qr_factor writes for this shape and options (the minimum
 * ldt): n for MIQR_T_FULL, the chosen top-level panel width for
 * MIQR_T_BLOCKED.  0 for invalid sizes or options.  Host only. */
int64_t qr_t_rows(int64_t m, int64_t n, const qr_opts *opts);

/* Description of the factorisation plan for this shape and options (lstsq
 * nonzero: the plan qr_lstsq uses), as JSON text: the tuning (b, bstar, nb,
 * leaf_rows, chain, arity, t_layout, lookahead; 0 for TSQR parameters chosen
 * per panel), the cost model's counts and predicted seconds, the workspace
 * regions in doubles, the recursion nodes [c0, rows, width, n1] (n1 = 0: a
 * TSQR panel) and the TSQR panels [c0, rows, width, leaf_rows, chain, arity,
 * levels].  Writes at most len - 1 characters and a NUL to buf (buf may be
 * NULL) and returns the full length, or -1 for invalid sizes or options.
 * Host only: needs no device. */
int64_t qr_plan(int64_t m, int64_t n, const qr_opts *opts, int lstsq, char *buf,
                int64_t len);

/* Flops (2 per multiply-add) of the GEMMs that the most recent qr_factor on
 * this handle launched: the algorithmic count of the EG updates, reported
 * beside the nominal 2mn^2 - 2n^3/3 (Alg. 2 forms the full T, which costs
 * more than the nominal count). */
double miqr_last_gemm_flops(miqr_handle handle);

/* Per-kernel timing.  While enabled (enable != 0, which also clears earlier
 * totals) every kernel the handle's entry points launch is bracketed by two
 * HIP events on its stream, and its algorithmic HBM bytes and flops are
 * recorded.  miqr_profile_kernels synchronises the pending events and returns
 * the number of distinct kernel names; miqr_profile_get reads entry `index`
 * (name copied into `name`, NUL-terminated, at most name_len bytes): total
 * milliseconds, launch count, total bytes and flops.  Any output pointer may
 * be NULL.  The events add a few microseconds per launch. */
miqr_status miqr_profile_enable(miqr_handle handle, int enable);
int miqr_profile_kernels(miqr_handle handle);
miqr_status miqr_profile_get(miqr_handle handle, int index, char *name,
                             int name_len, double *ms, int64_t *launches,
                             double *bytes, double *flops);

/* Launch graphs for qr_factor.  While enabled (enable != 0), qr_factor
 * records its launch sequence (the kernels of Alg. 2, its TSQR base cases of
 * Sec. 6.1 and the look-ahead stream's share, with their order) into a HIP
 * graph the first time it sees a key, and replays that graph as one launch on
 * the caller's stream on every later call with the same key.  The key is the
 * shape, the leading dimensions, the addresses of A, T, Q and sign_out, every
 * option and the handle's workspace address; a call with any of them
 * different is captured anew.  Replays run the same kernels in the same
 * order: results are bitwise those of the eager calls.  The buffers must stay
 * allocated while their graph may still be replayed (re-using an address for
 * a new buffer of the same shape is fine: the graph reads whatever is there
 * when it runs).  At most 64 graphs are kept per handle (all are dropped when
 * a 65th is captured, and when the workspace grows).  While per-kernel timing
 * (miqr_profile_enable) is on, calls run eagerly.  Disabling synchronises the
 * device and drops every graph.  miqr_graph_count returns the number kept.
 * Other entry points always launch eagerly. */
miqr_status miqr_graphs_enable(miqr_handle handle, int enable);
int64_t miqr_graph_count(miqr_handle handle);

/* QR factorisation in place (Alg. 2 with the TSQR base case of Sec. 6.1).
 *   A  (m x n, lda >= m, m >= n >= 1): on return R in the upper triangle and
 *      V's strict lower trapezoid below it.
 *   T  MIQR_T_FULL: n x n (ldt >= n), the full upper triangular kernel of
 *      Alg. 2's assembly, strict lower triangle set to zero.
 *      MIQR_T_BLOCKED: nb x n (ldt >= qr_t_rows), the panels' kernels (see
 *      miqr_t_layout).
 *   opts: see qr_opts; opts->Q (if set) receives the explicit thin Q.
 * With MIQR_T_BLOCKED and look-ahead the call also enqueues work on the
 * handle's internal stream, ordered after the caller's stream's earlier work
 * and joined back into it before the call's last operation.
 * Errors: MIQR_EINVAL (m < n, n < 1, lda < m, ldt too small, NULL A or T, an
 * option out of range, normalize without sign_out, Q with ldq < m),
 * MIQR_ENOMEM, MIQR_EHIP. */
miqr_status qr_factor(miqr_handle handle, void *stream, int64_t m, int64_t n,
                      double *A, int64_t lda, double *T, int64_t ldt,
                      const qr_opts *opts);

/* qr_factor for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as qr_factor, but every step runs on the
 * caller's stream (no look-ahead stream) and the workspace is a static 64 MiB
 * device array of the library, one per GPU, set up by miqr_create and held
 * until the process ends; the call allocates nothing.  Shapes whose
 * workspace does not fit (roughly m x n beyond 4e6 doubles of panel blocks;
 * qr_workspace_size reports the need without its split-K share) return
 * MIQR_EINVAL and enqueue nothing.  Every call on one GPU shares that array,
 * so calls that overlap on one GPU (different streams or threads, any handle)
 * race and must be ordered by the caller. */
miqr_status qr_factor_noalloc(miqr_handle handle, void *stream, int64_t m,
                              int64_t n, double *A, int64_t lda, double *T,
                              int64_t ldt, const qr_opts *opts);

/* Apply the orthogonal factor from qr_factor (Sec. 2.3, Q = I - V T V^T):
 *   trans 'N': C <- Q C;   trans 'T': C <- Q^T C.
 *   VR (m x n, lda) and T (n x n, ldt) as returned by qr_factor; C is m x k
 *   (ldc >= m), overwritten.  Evaluated right to left as three products
 *   (V^T C, then T or T^T, then C - V (.)), the order the paper states for the
 *   basis-kernel update.
 * Errors: MIQR_EINVAL (bad trans, m < n, k < 0, ld too small, NULL pointers). */
miqr_status qr_apply_q(miqr_handle handle, void *stream, char trans, int64_t m,
                       int64_t n, int64_t k, const double *VR, int64_t lda,
                       const double *T, int64_t ldt, double *C, int64_t ldc);

/* qr_apply_q for factors in the MIQR_T_BLOCKED layout with panel width nb
 * (T nb x n, ldt >= min(nb, n)): trans 'N': C <- Q_0 (Q_1 (... Q_{K-1} C)),
 * 'T': C <- Q_{K-1}^T (... Q_0^T C), each panel as three products.
 * Errors: as qr_apply_q, and nb < 1. */
miqr_status qr_apply_q_blocked(miqr_handle handle, void *stream, char trans,
                               int64_t m, int64_t n, int64_t k, const double *VR,
                               int64_t lda, const double *T, int64_t ldt,
                               int64_t nb, double *C, int64_t ldc);

/* Explicit thin Q = (I - V T V^T)[I_n; 0] (m x n, ldq >= m) from the factors.
 * If sign (device, n doubles) is non-NULL the columns are scaled by it
 * (Q D for factors computed with normalize). */
miqr_status qr_form_q(miqr_handle handle, void *stream, int64_t m, int64_t n,
                      const double *VR, int64_t lda, const double *T,
                      int64_t ldt, const double *sign, double *Q, int64_t ldq);

/* Least squares min ||B_j - A x_j||_2 for nrhs right-hand sides (the use that
 * motivates QR in Sec. 1).  A (m x n, m >= n) is overwritten by its factors;
 * B (m x nrhs, ldb >= m) by the solutions in rows 0..n-1 (LAPACK gels
 * convention).  FP64: factor, c = Q^T b, back substitution R x = c[0:n].
 * Mixed precisions: the factorisation runs with FP32/BF16 trailing updates and
 * the solution is refined in FP64 against a device copy of the original A
 * (R-preconditioned conjugate gradients on the normal equations, FP64
 * residuals) until the backward error is <= 1e-13 and has stopped
 * decreasing (at most 100 iterations, fewer when the observed contraction
 * cannot reach the gate in time); if the 1e-13 gate is not met the problem
 * is refactored in FP64 (info->fallback = 1, status MIQR_ENOCONV).
 *   info (host, may be NULL): when given, the call synchronises the stream and
 *   fills it.
 * Errors: MIQR_EINVAL, MIQR_ENOMEM, MIQR_EHIP, MIQR_ESINGULAR (some R_jj == 0
 * exactly; B is left holding Q^T b), MIQR_ENOCONV. */
miqr_status qr_lstsq(miqr_handle handle, void *stream, int64_t m, int64_t n,
                     int64_t nrhs, double *A, int64_t lda, double *B,
                     int64_t ldb, const qr_opts *opts, qr_info *info);

/* Solve with the triangular factor: X <- R^{-1} X for the n x n upper triangle
 * of VR (lda) and X (n x nrhs, ldx >= n).  Returns MIQR_ESINGULAR without
 * touching X if some R_jj == 0 (checked on the device; the call then
 * synchronises the stream). */
miqr_status qr_solve_r(miqr_handle handle, void *stream, int64_t n,
                       int64_t nrhs, const double *VR, int64_t lda, double *X,
                       int64_t ldx);

/* Backward error of least-squares solutions, the measure every least-squares
 * result of this library is gated on (the paper defines none):
 *   beta_j = ||A^T r_j||_2 / (||A||_F (||A||_F ||x_j||_2 + ||r_j||_2)),
 *   r_j = B[:, j] - A X[:, j],
 * zero exactly at a least-squares solution, computed in FP64 on the device
 * (the norms' quotients are taken before any product, so no product of norms
 * overflows).
 *   A (m x n, lda >= m), B (m x nrhs, ldb >= m), X (n x nrhs, ldx >= n):
 *   device, read only.  beta (host, nrhs doubles) receives the values, NaN
 *   where a norm's sum of squares overflows (entries of 1e154 and beyond);
 *   the mixed-precision solvers never accept such a value as converged.
 * Synchronises the stream.  Uses the handle's workspace.
 * Errors: MIQR_EINVAL (sizes, NULL pointers), MIQR_ENOMEM, MIQR_EHIP. */
miqr_status qr_backward_error(miqr_handle handle, void *stream, int64_t m, int64_t n,
                              int64_t nrhs, const double *A, int64_t lda,
                              const double *B, int64_t ldb, const double *X,
                              int64_t ldx, double *beta);

/* One problem of a batched least-squares call (device pointers). */
typedef struct qr_batch_item {
    int64_t m, n, nrhs; /* m >= n >= 1, 1 <= nrhs <= 8, n + nrhs <= 320 */
    double *A;          /* m x n, lda >= m; overwritten (R in the upper n x n
                           triangle, rows below it left as they were) */
    int64_t lda;
    double *B;          /* m x nrhs, ldb >= m; rows 0..n-1 receive X */
    int64_t ldb;
} qr_batch_item;

/* Many independent least-squares problems in persistent launches.  Each
 * problem is solved by one workgroup: Householder QR of the augmented matrix
 * [A | B] by a flat TSQR sweep over 64-row blocks (the TSQR of Sec. 5 /
 * App. C.1 with a chain as its reduction tree; dlarfg sign rule), the block's
 * reflectors applied sixteen at a time in the compact WY form of Sec. 2.3 on
 * MFMA, which leaves R and the top n rows of Q^T B, then back substitution.
 * Workgroups pop problems from device queues (one per register budget, by
 * n + nrhs), largest first.  A problem's arithmetic does not depend on the
 * other problems in the call, so its result is bitwise the same alone and in
 * any batch.
 *   items (host array of `count`): problems; pointers must not overlap.
 *   opts: NULL or precision MIQR_FP64, MIQR_MIXED_FP32 or MIQR_MIXED_BF16
 *   (other fields ignored; normalize and Q must be unset).  Mixed: the sweep
 *   runs on an FP32 working copy of each block with the two large products of
 *   every panel update on FP32 or BF16 MFMA (FP32 accumulation); reflector
 *   generation, T and R stay in FP64.  Each solution is then refined in FP64
 *   against the original A and B (R-preconditioned conjugate gradients on the
 *   normal equations, residual recomputed from A each iteration; with FP32
 *   products the first step is x += R^-1 R^-T A^T r) until every
 *   right-hand side's backward error (qr_backward_error's measure) is
 *   <= 1e-13 (the kernel aims at 5e-14, a margin for the rounding of its own
 *   estimate); a problem that does not get there within 40 iterations, or
 *   stops halving its error over four, is solved again in FP64.  Mixed
 *   precisions synchronise the stream.
 *   status (host, `count` int32, may be NULL): when given, the call
 *   synchronises the stream and writes 0, or j + 1 when R_jj == 0 exactly
 *   (that problem's B then holds the top n rows of Q^T B and A is unchanged).
 * Returns MIQR_ESINGULAR if status was given and some problem is singular.
 * Errors: MIQR_EINVAL (a bad item or precision; nothing is enqueued),
 * MIQR_ENOMEM, MIQR_EHIP (also when a bounded wait inside the kernel ran out,
 * an internal error: results are then not valid), MIQR_ENOTSUP. */
miqr_status qr_lstsq_batched(miqr_handle handle, void *stream, int64_t count,
                             const qr_batch_item *items, const qr_opts *opts,
                             int32_t *status);

/* qr_lstsq_batched with, per item, the refinement iterations of a mixed
 * precision: iters (host, `count` int32, may be NULL) receives 0 for FP64,
 * the FP64 refinement iterations that met the target, or -1 for a problem
 * solved again in FP64.  Synchronises the stream when status or iters is
 * given. */
miqr_status qr_lstsq_batched_ex(miqr_handle handle, void *stream, int64_t count,
                                const qr_batch_item *items, const qr_opts *opts,
                                int32_t *status, int32_t *iters);

/* ---- Serving loop -------------------------------------------------------
 * A least-squares server on one device.  Requests (host matrices) wait in
 * arrival order until device memory for them fits in the HBM budget; then
 * their upload starts on a copy stream.  Uploaded requests are packed into
 * batches solved by the batched kernel of qr_lstsq_batched, one captured-graph
 * replay per batch, with up to two batches in flight: requests that arrive
 * while a batch runs join the next one (continuous batching), and their
 * uploads overlap the running batch.  A request's result is bitwise the same
 * whatever it is batched with.  The caller drives the server with
 * qr_server_poll; the server is not thread-safe.  Host buffers passed to
 * submit/resolve must stay valid and unchanged until the request is reported
 * done; pinned host memory lets uploads overlap compute. */
typedef struct miqr_server *miqr_server_handle;

typedef struct qr_server_opts {
    int64_t hbm_budget;   /* device bytes for admitted requests (0: 8 GiB) */
    int64_t max_batch;    /* requests per launch (0: 4096) */
    int64_t max_pending;  /* waiting requests before submit says MIQR_EBUSY
                             (0: 2^20) */
    int64_t stage_bytes;  /* per in-flight batch, solution staging (0: 64 MiB) */
    int32_t keep_factors; /* nonzero: each factorisation stays on the device
                             for qr_server_resolve until qr_server_release
                             (FP64 only) */
    int32_t precision;    /* MIQR_FP64 (0), MIQR_MIXED_FP32 or MIQR_MIXED_BF16:
                             as for qr_lstsq_batched; a request whose
                             refinement misses 1e-13 is solved again in FP64
                             in a later batch */
} qr_server_opts;

typedef struct qr_server_done {
    int64_t id;
    int32_t status;     /* 0, or j + 1 if R_jj == 0 (X then holds the top n
                           rows of Q^T B) */
    int32_t batch_size; /* requests in the launch that served it */
    double submit_s;    /* server clock, seconds: submission */
    double start_s;     /* launch of its batch */
    double end_s;       /* completion observed by qr_server_poll */
} qr_server_done;

/* Create a server on the handle's device (allocates the HBM budget, two batch
 * slots and their captured graphs).  The handle must outlive the server. */
miqr_status qr_server_create(miqr_handle handle, const qr_server_opts *opts,
                             miqr_server_handle *server);
/* Wait for in-flight work and free everything the server holds. */
miqr_status qr_server_destroy(miqr_server_handle server);
/* Seconds on the server's clock (the clock of qr_server_done). */
double qr_server_clock(miqr_server_handle server);
/* Queue min ||B - A X||: A (host, m x n, lda), B (host, m x nrhs, ldb); X
 * (host, n x nrhs, ldx) receives the solution.  Limits as qr_batch_item.
 * MIQR_EBUSY when max_pending requests are already waiting; MIQR_EINVAL for a
 * request that cannot fit the budget even alone. */
miqr_status qr_server_submit(miqr_server_handle server, int64_t m, int64_t n,
                             int64_t nrhs, const double *A, int64_t lda,
                             const double *B, int64_t ldb, double *X,
                             int64_t ldx, int64_t *id);
/* Queue further right-hand sides against a finished request whose
 * factorisation was kept (keep_factors): only B is uploaded; the stored
 * reflectors are replayed on it, then back substitution. */
miqr_status qr_server_resolve(miqr_server_handle server, int64_t factored_id,
                              int64_t nrhs, const double *B, int64_t ldb,
                              double *X, int64_t ldx, int64_t *id);
/* Drop a kept factorisation (MIQR_EBUSY while solves against it run). */
miqr_status qr_server_release(miqr_server_handle server, int64_t factored_id);
/* Retire finished batches (copying solutions into the callers' X), admit
 * waiting requests, launch batches into free slots, then report up to
 * `capacity` finished requests.  wait != 0 blocks until at least one request
 * is finished, unless nothing is queued or in flight. */
miqr_status qr_server_poll(miqr_server_handle server, int wait,
                           qr_server_done *done, int64_t capacity,
                           int64_t *ndone);
/* Requests waiting, uploaded but not launched, and running; device bytes in
 * use.  Any pointer may be NULL. */
miqr_status qr_server_stats(miqr_server_handle server, int64_t *pending,
                            int64_t *admitted, int64_t *running,
                            int64_t *hbm_used);

#ifdef __cplusplus
}
#endif

#endif /* MIQR_H */
