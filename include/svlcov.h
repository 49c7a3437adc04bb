/*
 * svlcov.h -- C ABI of an MI355X (gfx950) engine that keeps a rank-k truncated
 * SVD  A ~= U diag(sigma) V^T  of a sparse, evolving matrix up to date under
 * the three update forms of arXiv 2401.09703 (Section 2):
 *
 *     add rows        [A ; E_r]            E_r  s x n
 *     add columns     [A , E_c]            E_c  m x s   (passed as E_c^T, s x m)
 *     update weights  A + D E_m^T          D    m x s   (passed as D^T,  s x m)
 *                                          E_m  n x s   (passed as E_m^T, s x n)
 *
 * Each update maintains an approximate rank-k truncated SVD in the sense of
 * Definition 2: the new factors are SVD_k of the update applied to
 * U diag(sigma) V^T (Theorem 1).  The factors are held in the extended
 * decomposition of Section 3.2, U = U_base W_U and V = V_base W_V with W_U,
 * W_V k x k, so that an update touches only the rows of the tall factors that
 * the update's sparsity reaches plus the appended rows.
 *
 * Every update runs on the GPU: the projection of the update onto the tall
 * factor (Lemma 1), the Gram of the augmented matrix without forming it
 * (Lemma 2, Lemma 3), its FP64 Cholesky factor (the R of Algorithm 2), the
 * (k+s) Rayleigh-Ritz SVD (Section 2.1, step 2), the k x k factor updates and
 * the sparse row updates of the tall factors (Equation (1); Algorithms 3, 4
 * and 11).
 *
 * Conventions
 *   - Matrices are row-major unless stated.  Sparse inputs are canonical CSR:
 *     0-based, int64 row_ptr[rows+1] with row_ptr[0] = 0 and row_ptr[rows] =
 *     nnz, int32 column ids strictly increasing within each row, finite
 *     values (explicit zeros allowed, empty rows allowed).
 *   - Ownership: the caller owns every input pointer.  Host inputs are read
 *     before the call returns.  Device inputs must stay valid until the next
 *     svlcov_sync() on the same state.  The state owns all device memory it
 *     allocates (factors and workspaces).
 *   - Streams: all device work of a state is ordered on the stream given in
 *     svlcov_options (NULL = a stream the library creates).  Update calls are
 *     asynchronous; svlcov_sync() waits and reports deferred errors.  Device
 *     inputs are read on that stream with no other ordering: work on another
 *     stream that produces them must be complete, or the state's stream must
 *     wait for it (an event recorded after the producer, hipStreamWaitEvent
 *     on svlcov_stream()), before the update call.
 *   - Memory: the state allocates its factors and workspaces through the
 *     dev_alloc / dev_free hooks of svlcov_options when both are given (so a
 *     framework's allocator can own them), else with hipMallocAsync /
 *     hipFreeAsync on the state's stream.
 *   - Errors: return codes only, nothing is thrown or printed across the ABI.
 *     A call that fails validation on the host leaves the state unchanged.  A
 *     failure found on the device (malformed device-resident CSR, non-finite
 *     intermediate) makes every remaining kernel of that update and of later
 *     updates a no-op, so the factors stay as they were before the failing
 *     update; the error is returned by the next svlcov_sync(), which also
 *     restores the row/column counts to their values before that update.
 *   - Threads: one state must not be used from two threads at once
 *     (SVLCOV_E_BUSY is returned to the second caller).
 */
#ifndef SVLCOV_H
#define SVLCOV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct svlcov_state svlcov_state;

typedef enum {
  SVLCOV_OK = 0,
  SVLCOV_E_INVALID = 1,     /* malformed argument or CSR                      */
  SVLCOV_E_SHAPE = 2,       /* dimensions do not match the state              */
  SVLCOV_E_NOMEM = 3,       /* device allocation failed                       */
  SVLCOV_E_NUMERIC = 4,     /* non-finite input or intermediate               */
  SVLCOV_E_DEVICE = 5,      /* HIP runtime error                              */
  SVLCOV_E_BUSY = 6,        /* state in use by another thread                 */
  SVLCOV_E_UNSUPPORTED = 7  /* size or option outside what is built           */
} svlcov_status;

typedef enum {
  SVLCOV_FP64 = 0,    /* all storage and arithmetic FP64                       */
  SVLCOV_FP32 = 1,    /* FP32 tall factors, FP32 SpMM/GEMM; FP64 small dense    */
  SVLCOV_BF16X3 = 2   /* as FP32, but the residual Gram and the realisation    */
                      /* GEMMs run as three BF16 MFMA products (hi*hi + hi*lo  */
                      /* + lo*hi) with FP32 accumulation                       */
} svlcov_precision;

typedef enum { SVLCOV_F32 = 0, SVLCOV_F64 = 1 } svlcov_dtype;

typedef struct {
  int64_t rows, cols, nnz;
  const int64_t *row_ptr;   /* rows + 1 */
  const int32_t *col_idx;   /* nnz      */
  const void *val;          /* nnz, float or double per val_dtype */
  int32_t val_dtype;        /* svlcov_dtype */
  int32_t on_device;        /* 0: host memory, 1: device memory of the state */
} svlcov_csr;

typedef struct {
  int32_t precision;          /* svlcov_precision                              */
  int32_t device;             /* HIP device ordinal                            */
  void *stream;               /* hipStream_t, NULL = library-created stream    */
  int64_t row_capacity;       /* initial row capacity of U_base (>= m), 0=auto */
  int64_t col_capacity;       /* initial row capacity of V_base (>= n), 0=auto */
  double rank_tol;            /* relative pivot floor of the residual Gram     */
                              /* Cholesky (drop when d_j <= rank_tol * max_i   */
                              /* ||e_i||^2); <= 0 selects the mode's default   */
  double cond_reset;          /* fold W into the tall factor when its 1-norm   */
                              /* condition number exceeds this (default 1e4 in */
                              /* FP64, 1e2 in FP32 and BF16X3); <= 0 default   */
  int32_t validate_device_inputs; /* 1: check device CSR on the device         */
  /* Device allocator hooks (both or neither; NULL = hipMallocAsync /
   * hipFreeAsync).  dev_alloc returns bytes of device memory of the state's
   * device that may be used by work enqueued on `stream` (the state's stream)
   * from the moment it returns, or NULL on failure (SVLCOV_E_NOMEM).
   * dev_free releases a block from dev_alloc; work already enqueued on
   * `stream` may still use it, so it may be reused only by work ordered
   * after that (a stream-ordered caching allocator satisfies this).  Both are
   * called from the thread of the state's call (one of a request server's
   * dispatch threads for attached states), never concurrently for one state. */
  void *(*dev_alloc)(size_t bytes, void *stream, void *ctx);
  void (*dev_free)(void *ptr, size_t bytes, void *stream, void *ctx);
  void *alloc_ctx;              /* passed to both hooks                          */
  int32_t deterministic;        /* 1 (default): the sparse row update sums each  */
                                /* base row's terms in a fixed order (nonzeros   */
                                /* sorted by column, no floating-point atomics), */
                                /* so an update gives bitwise the same factors   */
                                /* every time; 0: atomic accumulation, faster,   */
                                /* rounding order free                           */
  int32_t side_stream;          /* 1 (default): an append update (FP32/BF16X3,   */
                                /* k+32 rounded to 16 at most 160) runs the      */
                                /* residual Gram's Cholesky and K, later one     */
                                /* side's k x k update, on a second stream of    */
                                /* the state beside the eigensolver; that work   */
                                /* is ordered after the call's earlier work on   */
                                /* `stream` and before its later work there, so  */
                                /* the state's stream still orders everything;   */
                                /* the factors are bitwise those of 0 (one       */
                                /* stream)                                       */
} svlcov_options;

typedef struct {
  int64_t updates;            /* completed update calls                        */
  int64_t resets_U, resets_V; /* times W_U / W_V was folded into the base      */
  int32_t last_rank;          /* kept pivots of the last orthogonalisation     */
  int32_t last_rank2;         /* second side of a weight update (else -1)      */
  double last_kappa_U;        /* 1-norm condition estimate of W_U after last   */
  double last_kappa_V;        /*   update (before any reset)                   */
  double last_min_kept_pivot; /* smallest kept / largest dropped pivot ratio   */
  double last_max_dropped_pivot; /* relative to max ||e_i||^2 (-1 if none)     */
  int64_t iter_runs;          /* eigenproblems solved by the iterative solver  */
  int64_t iter_steps;         /*   its filter steps in total                   */
  int64_t iter_fallbacks;     /*   runs handed to the direct solver            */
  double iter_flops;          /*   its algorithmic flops (products with M)     */
} svlcov_stats;

/* Fill *opt with defaults: FP64, device 0, library stream, automatic
 * capacities, default tolerances, device-input validation on. */
void svlcov_default_options(svlcov_options *opt);

/* Create a state holding m x k U, k sigma, n x k V (FP64, row-major, host
 * memory if factors_on_device == 0, else device memory).  U and V must have
 * orthonormal columns and sigma must be non-increasing and >= 0: these are
 * the starting factors U', V' of the extended decomposition with U'' = V'' =
 * I (Section 3.2).  k must be one of 16, 32, 64, 128. */
svlcov_status svlcov_init(svlcov_state **out, int64_t m, int64_t n, int32_t k,
                          const double *U, const double *sigma, const double *V,
                          int32_t factors_on_device, const svlcov_options *opt);

/* Add rows: E_r is s x n (Algorithm 11; Theorem 1, add rows).  m grows by s. */
svlcov_status svlcov_add_rows(svlcov_state *h, const svlcov_csr *E_r);

/* Add columns: E_c_T is s x m, the transpose of the new columns (Algorithm 3;
 * Theorem 1, add columns).  n grows by s. */
svlcov_status svlcov_add_cols(svlcov_state *h, const svlcov_csr *E_c_T);

/* Update weights: A + D E_m^T with D_T s x m and E_m_T s x n (Algorithm 4;
 * Theorem 1, update weights).  Both must have the same number of rows s. */
svlcov_status svlcov_update_weights(svlcov_state *h, const svlcov_csr *D_T,
                                    const svlcov_csr *E_m_T);

/* The -GKL and -RPI variants (the appendix on approximating the augmented
 * space; the variants paragraph of Section 4).  The augmented matrix
 * Z = (I - V V^T) E_r^T (rows) or (I - U U^T) E_c (columns) is replaced by
 * an l-dimensional orthonormal basis Q of a subspace of its range together
 * with P = Z^T Q, so that the Rayleigh-Ritz problem has k + l columns on that
 * side instead of k + s; everything else is the update of svlcov_add_rows /
 * svlcov_add_cols.  Q never exists: it is kept as coefficients Y (q = Z y)
 * and every product with Z or Z^T goes through the residual Gram Z^T Z.
 *   method  SVLCOV_APPROX_GKL: Golub-Kahan-Lanczos from the start vector p_1
 *           (start: s doubles of nonzero norm, normalised here; NULL = all
 *           ones), every new p orthogonalised against all previous ones; a
 *           coefficient whose square falls to rank_tol times the largest
 *           squared row norm of the update stops the process (the rest of
 *           the basis is zero).
 *           SVLCOV_APPROX_RPI: t rounds of P <- orth(P), Q <- orth(Z P),
 *           P <- Z^T Q from the start P_0 (start: l vectors of s doubles,
 *           vector j at start[j * s]; required); directions whose pivot
 *           falls to the same threshold are dropped.
 *   l       1 <= l <= 64, clamped to s; RPI reads min(l, s) start vectors.
 *   t       RPI rounds, 1 <= t <= 16 (ignored by GKL).
 *   start_on_device  0: host memory (read before the call returns),
 *           1: device memory of the state (valid until the next sync).
 * Errors as for svlcov_add_rows, and SVLCOV_E_INVALID for a bad method, l,
 * t or a missing RPI start; SVLCOV_E_NUMERIC for a non-finite host start. */
typedef enum { SVLCOV_APPROX_GKL = 1, SVLCOV_APPROX_RPI = 2 } svlcov_approx_method;
typedef struct {
  int32_t method;            /* svlcov_approx_method                          */
  int32_t l;                 /* dimension of the approximate space            */
  int32_t t;                 /* RPI rounds                                    */
  int32_t start_on_device;   /* 0 host, 1 device                              */
  const double *start;       /* p_1 (GKL, may be NULL) or P_0 (RPI)           */
} svlcov_approx;
svlcov_status svlcov_add_rows_approx(svlcov_state *h, const svlcov_csr *E_r,
                                     const svlcov_approx *a);
svlcov_status svlcov_add_cols_approx(svlcov_state *h, const svlcov_csr *E_c_T,
                                     const svlcov_approx *a);
/* The same variants for the weight form A + D E_m^T (the appendix's weight
 * algorithm): a_D gives the method, l, t and start of the basis of the
 * augmented space of D against U, a_E those of E_m against V (the two may
 * differ); K = [[Sigma, 0], [0, 0]] + [U^T D ; P_D^T] [V^T E_m ; P_E^T]^T is
 * (k + l_D) x (k + l_E), each l clamped to s.  Arguments, errors and the
 * asynchronous behaviour are those of svlcov_update_weights. */
svlcov_status svlcov_update_weights_approx(svlcov_state *h, const svlcov_csr *D_T,
                                           const svlcov_csr *E_m_T, const svlcov_approx *a_D,
                                           const svlcov_approx *a_E);

/* Realise and return the factors U = U_base W_U (m x k), sigma (k) and
 * V = V_base W_V (n x k).  Any output pointer may be NULL; m, n, k receive the
 * current shape when non-NULL.  out_dtype selects float or double outputs,
 * out_on_device selects device or host output buffers.  Waits for the state's
 * stream. */
svlcov_status svlcov_get_factors(svlcov_state *h, int64_t *m, int64_t *n,
                                 int32_t *k, int32_t out_dtype,
                                 int32_t out_on_device, void *U, double *sigma,
                                 void *V);

/* Query(i) of Theorem 1: row i of U (side 0) or of V (side 1) as
 * U_base[i] W_U in O(k^2); writes k doubles to host memory. */
svlcov_status svlcov_query_row(svlcov_state *h, int32_t side, int64_t i,
                               double *out_k);

/* Query(i) of Theorem 1 for many rows at once: out (device, n x k FP64,
 * row-major) receives row idx[r] of U (side 0) or V (side 1) formed as
 * base[idx[r]] W in O(k^2) each.  idx is device int64; rows with an index
 * outside the factor are NaN.  Asynchronous on the state's stream. */
svlcov_status svlcov_query_rows(svlcov_state *h, int32_t side, int64_t n, const int64_t *idx,
                                double *out);

/* The pair score of the link-prediction and collaborative-filtering
 * workloads (Section 5): out[p] = U[i_p]^T Sigma V[j_p]; with both = 1 the
 * larger of that and U[j_p]^T Sigma V[i_p] (undirected graphs; both indices
 * must then lie in both factors).  i, j are device int64, out device FP64
 * (n each); a pair outside the factors scores NaN.  The factors are realised
 * once per factor version as U_base (W_U Sigma) and V_base W_V in the storage
 * type (FP32 products for the FP32 and BF16x3 modes) and kept on the state
 * until its next update; each pair is then two row gathers and a k-term dot
 * product (four gathers with both).  Asynchronous on the state's stream;
 * with kernel_ms non-NULL the call waits and reports the scoring kernel's
 * device time. */
svlcov_status svlcov_score_pairs(svlcov_state *h, int64_t n, const int64_t *i, const int64_t *j,
                                 int32_t both, double *out, float *kernel_ms);

/* Wait for all work queued on the state and report a deferred error. *//* Wait for all work queued on the state and report a deferred error. */
svlcov_status svlcov_sync(svlcov_state *h);

/* Counters and the numerical diagnostics of the last update (waits). */
svlcov_status svlcov_get_stats(svlcov_state *h, svlcov_stats *out);

/* Diagnostics.  With profiling enabled, every phase of an update is bracketed
 * by HIP events on the state's stream; svlcov_phase_times() waits, then adds
 * the elapsed milliseconds and the number of occurrences of each phase since
 * the previous call into ms[0..n) and count[0..n) (either may be NULL).  The
 * phases are, in order: validate, spmm_w, sparse_gram, resid_gram, cholesky,
 * build_K, kkt_gemm, tridiag, bisect, stein, backtransform, recover_G,
 * orthonormalize, small_factor, trsm, commit, subspace_iter (the iterative
 * eigensolver of the FP32 / BF16x3 modes, which replaces tridiag .. 
 * backtransform unless it falls back to them). */
#define SVLCOV_NUM_PHASES 17
svlcov_status svlcov_profile(svlcov_state *h, int32_t enable);
/* Profiling of some phases only: bit i of mask (phases numbered as
 * svlcov_phase_name numbers them) times phase i; mask 0 turns profiling
 * off, and svlcov_profile(h, 1) is the mask of every phase.  Each timed
 * occurrence of a phase records two events on the state's stream, host
 * work that can hold up the launches of a short update, so a timed run
 * that needs one phase's duration times that phase alone.  Bits at or
 * above SVLCOV_NUM_PHASES: SVLCOV_E_INVALID. */
svlcov_status svlcov_profile_phases(svlcov_state *h, uint32_t mask);
svlcov_status svlcov_phase_times(svlcov_state *h, double *ms, int64_t *count, int32_t n);
const char *svlcov_phase_name(int32_t i);

/* Tile shapes of the fused projection (svlcov_project_batch and the request
 * server's fused launches): variant v gathers with loads_in_flight 16-byte
 * loads per lane and takes rows_per_tile rows of an update per workgroup.
 * The shape used for an update is looked up in a process-wide table by
 * (fp64: 1 for FP64 storage, 0 for FP32; the rank k in 16/32/64/128; the
 * row bin of its mean nonzeros per row: 0 below 16, 1 below 64, 2 below 256,
 * 3 otherwise).  Every entry starts at variant 0; the tuner writes the
 * measured best ones.  These calls touch no device.  Errors: SVLCOV_E_INVALID
 * for a variant or key out of range or a NULL output. */
int32_t svlcov_spmm_variant_count(void);
svlcov_status svlcov_spmm_variant_shape(int32_t v, int32_t *loads_in_flight,
                                        int32_t *rows_per_tile);
svlcov_status svlcov_spmm_tune_set(int32_t fp64, int32_t k, int32_t row_bin, int32_t variant);
svlcov_status svlcov_spmm_tune_get(int32_t fp64, int32_t k, int32_t row_bin, int32_t *variant);

/* Building block of the (k+s) Rayleigh-Ritz SVD (Section 2.1, step 2): the k
 * largest eigenpairs of the symmetric N x N FP64 matrix M (row-major, device
 * memory, not modified).  lam (device, k doubles) receives the eigenvalues in
 * non-increasing order, vecs (device, k x N row-major) the eigenvectors, one
 * per row, sign fixed so that the entry of largest magnitude is positive.
 * Workspace is allocated and freed on `stream` (hipStream_t, NULL = default
 * stream).  N <= 6144 and k <= 128. */
svlcov_status svlcov_sym_eig_topk(int64_t N, const double *M, int32_t k, double *lam,
                                  double *vecs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation, arguments and results as svlcov_sym_eig_topk, with no
 * allocation at all.  The workspace (a copy of M, the eigensolver's work
 * arrays, its status word and barrier flags) lives in one library-owned
 * device array of SVLCOV_EIG_SCRATCH_BYTES per GPU, set up on the first call
 * on that device and held until the process ends.  The call only enqueues
 * work on `stream` (hipStream_t, NULL = default stream) and does not wait.
 * SVLCOV_E_UNSUPPORTED when the workspace of (N, k), 8 (N^2 + 7N + 7Nk) bytes
 * plus about 8 KiB per 32 rows and 17 KiB of flags, exceeds the array
 * (N up to about 1500 at k = 64), as well as for N > 6144 or k > 128;
 * SVLCOV_E_INVALID for bad arguments.  Every call on one GPU shares that
 * GPU's array and leaves its contents behind (the status word and flags are
 * cleared at the start of each call): calls that overlap on one GPU, from two
 * streams or two threads, race and must be serialised by the caller. */
#define SVLCOV_EIG_SCRATCH_BYTES (24u << 20)
svlcov_status svlcov_sym_eig_topk_noalloc(int64_t N, const double *M, int32_t k, double *lam,
                                          double *vecs, void *stream);

/* Initial rank-k truncated SVD of a sparse m x n matrix A, the starting
 * factors U', sigma, V' that every experiment of Section 5 updates from (the
 * paper leaves their computation to the randomised methods its introduction
 * cites).  The randomised range finder with `power` subspace iterations
 * (Halko, Martinsson and Tropp 2011, Algorithms 4.4 and 5.1):
 *     Q = orth(A Omega);  repeat power times: Q = orth(A orth(A^T Q));
 *     B = Q^T A = U_B diag(sigma_B) V_B^T;  U = Q U_B[:, :k],
 *     sigma = sigma_B[:k],  V = V_B[:, :k].
 * A: canonical CSR (host or device memory per on_device; FP32 or FP64
 * values); checked on the device, SVLCOV_E_INVALID if malformed.
 * Omega: the n x l Gaussian test matrix (device, FP64 row-major), drawn by
 * the caller, so that the result is a deterministic function of (A, Omega).
 * l in {16, 32, 64, 128} (SVLCOV_E_UNSUPPORTED otherwise), 1 <= k <= l,
 * l <= min(m, n) (SVLCOV_E_SHAPE), 0 <= power <= 64, nnz < 2^31.
 * Outputs (device, FP64 row-major, caller-owned): U m x k, sigma k
 * (non-increasing), V n x k; U and V have orthonormal columns to rounding.
 * Singular values below 1e-7 sigma_0 are not resolved by the l x l Gram:
 * their vectors are an orthonormal completion.  phase_ms (host, NULL for
 * none) receives SVLCOV_RSVD_PHASES times in ms: transpose and validation,
 * products with A and A^T, orthonormalisations, the l x l eigenproblem, the
 * final products.  Workspace (about 16 (m + n) l + 40 nnz bytes) is allocated
 * and freed on `stream` (hipStream_t, NULL = default stream); the call
 * returns after the stream has finished the work.  Non-finite values in
 * Omega give SVLCOV_E_NUMERIC. */
#define SVLCOV_RSVD_PHASES 5
svlcov_status svlcov_rsvd(const svlcov_csr *A, int32_t k, int32_t l, int32_t power,
                          const double *Omega, double *U, double *sigma, double *V,
                          double *phase_ms, void *stream);

/* ------------------------------------------------------------------------
 * Request server (continuous batching of updates over many matrices).
 *
 * A server keeps the factors of many matrices resident on one GPU and runs
 * their update requests (the three forms above) as they arrive.  A scheduler
 * thread admits requests in arrival order whenever one of max_inflight slots
 * is free and the device workspace of the admitted requests stays within
 * workspace_budget bytes (a request's footprint is the exact workspace its
 * update carves, plus staging for host inputs; a request larger than the
 * budget is admitted alone).  Requests of one matrix run one at a time in
 * submission order; requests of different matrices run on their own streams
 * and overlap on the device.  The projections (C' = E base W, the first step)
 * of all requests admitted together whose inputs are device-resident and not
 * re-validated on the device run as one fused launch.  Cooperative kernels of
 * different requests are ordered one after another (each needs all of its
 * blocks resident).  Each
 * request's result equals the result of the same update applied alone, up
 * to the rounding of floating-point atomics.
 * ---------------------------------------------------------------------- */
typedef struct svlcov_server svlcov_server;

typedef struct {
  int32_t device;             /* HIP device ordinal (= the attached states')   */
  int32_t max_inflight;       /* concurrent requests, 1..64                    */
  int64_t workspace_budget;   /* bytes of device workspace for in-flight       */
                              /* requests; <= 0 selects 8 GiB                  */
} svlcov_server_options;

typedef struct {
  int64_t submitted, completed, failed;
  int64_t peak_inflight;          /* most requests in flight at once          */
  int64_t peak_workspace_bytes;   /* largest admitted workspace sum           */
  int64_t fused_launches;         /* fused projection launches                */
  int64_t fused_requests;         /* requests whose projection was fused      */
  double fused_ms;                /* device time of those launches            */
} svlcov_server_stats;

void svlcov_server_default_options(svlcov_server_options *opt);
svlcov_status svlcov_server_create(svlcov_server **out, const svlcov_server_options *opt);

/* Hand a state (from svlcov_init, idle) to the server; from now on only the
 * server may update it (svlcov_get_factors / svlcov_query_row are fine once
 * svlcov_server_drain has returned).  Its own update workspaces are freed:
 * requests borrow a slot's.  *matrix_id receives the id used by submit. */
svlcov_status svlcov_server_attach(svlcov_server *srv, svlcov_state *h, int32_t *matrix_id);

/* Queue one update: op 0 add rows (A = E_r), 1 add columns (A = E_c^T),
 * 2 update weights (A = D^T, B = E_m^T).  Host CSR inputs are copied before
 * the call returns; device CSR inputs must stay valid until the request
 * completes.  Shape and format errors are reported as the request's result. */
svlcov_status svlcov_server_submit(svlcov_server *srv, int32_t matrix_id, int32_t op,
                                   const svlcov_csr *A, const svlcov_csr *B, int64_t *ticket);

/* Result of a request: *result is its status (as the direct call would
 * return it, device-side failures included), *latency_ms the time from
 * submit to completion.  wait blocks; poll sets *done = 0 while it runs.  A
 * ticket is forgotten once its result has been returned. */
svlcov_status svlcov_server_wait(svlcov_server *srv, int64_t ticket, svlcov_status *result,
                                 double *latency_ms);
svlcov_status svlcov_server_poll(svlcov_server *srv, int64_t ticket, int32_t *done,
                                 svlcov_status *result, double *latency_ms);

/* Wait until every submitted request has completed. */
svlcov_status svlcov_server_drain(svlcov_server *srv);
svlcov_status svlcov_server_get_stats(svlcov_server *srv, svlcov_server_stats *out);

/* Drain, stop the scheduler, and give the attached states back to the caller
 * (they are not destroyed). */
void svlcov_server_destroy(svlcov_server *srv);

/* The projection C' = E base W of many updates in one launch (the first
 * step of an update, Lemma 1; the fused form the request server uses).
 * Item i projects E[i] (device CSR; width m of states[i] for side 0, n for
 * side 1) on U_base W_U (side 0) or V_base W_V (side 1) of states[i], writing
 * C' (E[i].rows x k FP64, row-major, device) to out[i] and the squared row
 * norms of E[i] to rown[i] (device, may be NULL).  The states must be idle
 * (synced) and on one device; the launch runs on `stream` and the call waits
 * for it.  kernel_ms (may be NULL) receives the launch's device time. */
svlcov_status svlcov_project_batch(int32_t n, svlcov_state *const *states, const int32_t *sides,
                                   const svlcov_csr *E, double *const *out, double *const *rown,
                                   void *stream, float *kernel_ms);

/* The hipStream_t the state enqueues on. */
void *svlcov_stream(svlcov_state *h);

/* Release the state and all device memory it holds (after waiting for its
 * stream).  A call in flight on the state from another thread finishes
 * first.  A state attached to a request server is not released (the call
 * returns without effect): destroy the server first. */
void svlcov_destroy(svlcov_state *h);

const char *svlcov_status_str(svlcov_status s);

#ifdef __cplusplus
}
#endif
#endif /* SVLCOV_H */
