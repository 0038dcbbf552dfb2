/*
 * lanczos_topk.h -- C ABI of the MI355X (gfx950) Top-K sparse symmetric
 * eigensolver: Lanczos with full reorthogonalisation, a Jacobi eigensolve of
 * the tridiagonal matrix and the Ritz-vector product.
 *
 * Method: Sgherzi, Parravicini, Santambrogio, "A Mixed Precision, Multi-GPU
 * Design for Large-scale Top-K Sparse Eigenproblems" (2022).
 *   Sec. III, Algorithm 1   Lanczos iteration (SpMV, alpha, three-term update,
 *                           orthogonalisation, beta, normalisation)
 *   Sec. III (2nd phase)    Jacobi on the tridiagonal T, Ritz vectors V*S
 *   Sec. I                  Top-K = the K eigenvalues largest in modulus
 *   Sec. III-A              storage vs. computation precision (FDF)
 *   Sec. III-B, IV-B        out-of-core matrices (host-resident mode)
 *   Sec. IV-D               accuracy metrics: L2 residual, pairwise angle
 *
 * Conventions shared by every entry point:
 *   - Return value is an lz_status code; it is the only error channel.
 *   - Argument errors are detected before anything is enqueued.
 *   - Device pointers are HIP device allocations owned by the caller; the
 *     library never frees them.  `stream` is a hipStream_t passed as void*
 *     (NULL = the default stream); work is enqueued on it.
 *   - CSR input: rowptr int64[n+1] with rowptr[0] = 0 and non-decreasing,
 *     col int32[nnz] with 0 <= col < n (any order within a row), val[nnz] in
 *     the storage precision: double (LZ_FP64), float (LZ_FP32) or bfloat16
 *     bits as uint16 (LZ_BF16).  The matrix must be symmetric (caller's
 *     contract; not checked).
 *   - Limits: n >= 1, 1 <= K <= m <= min(n, LZ_MAX_STEPS), n < 2^31.
 */
#ifndef LANCZOS_TOPK_H
#define LANCZOS_TOPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LZ_MAX_STEPS 64

/* Storage precision of the matrix values and the Lanczos basis (Sec. III-A).
 * LZ_FP64: values, basis and SpMV accumulation in binary64.
 * LZ_FP32: values and basis stored binary32, SpMV accumulates in binary32.
 * LZ_BF16: values and basis stored bfloat16, SpMV accumulates in binary32.
 * In every mode alpha/beta, the reorthogonalisation coefficients, the Jacobi
 * solve, the Ritz product and the residual report are binary64. */
typedef enum { LZ_FP64 = 0, LZ_FP32 = 1, LZ_BF16 = 2 } lz_precision;

typedef enum {
    LZ_OK = 0,
    LZ_ERR_INVALID_ARG = -1,        /* null pointer, bad size or precision */
    LZ_ERR_OUT_OF_MEMORY = -2,      /* library-side allocation failed */
    LZ_ERR_HIP = -3,                /* a HIP runtime call failed */
    LZ_ERR_WORKSPACE_TOO_SMALL = -4,
    LZ_ERR_TOO_LARGE = -5,          /* serving: request exceeds the HBM budget */
    LZ_ERR_NOT_CONVERGED = -6,      /* Jacobi hit its sweep limit */
    LZ_ERR_NONFINITE = -7,          /* NaN or Inf appeared in beta */
    LZ_ERR_BREAKDOWN = -8,          /* a restart vector had no component
                                       outside the basis */
    LZ_ERR_RESTART_BUDGET = -9,     /* stream-ordered call: more breakdowns
                                       than lz_options.max_restarts */
    LZ_PENDING = 1                  /* serving: request not finished yet */
} lz_status;

/* Reorthogonalisation modes (Algorithm 1, orthogonalisation loop). */
#define LZ_REORTH_NONE 0       /* three-term recurrence only */
#define LZ_REORTH_ONCE 1       /* one classical Gram-Schmidt pass */
#define LZ_REORTH_TWICE 2      /* two passes ("twice is enough"); default */
#define LZ_REORTH_SELECTIVE 3  /* second pass only when its correction
                                  exceeds the storage rounding of w */

/* Row order of the solve.  Algorithm 1 applied to P A P^T (P a permutation)
   has the same Ritz values, and its Ritz vectors are P y; the library may
   relabel the rows and columns of the matrix hub-first (a stable sort by
   degree class, longest rows first) so that the gathers of the SpMV hit a
   compact, cached part of the vector.  Start and restart vectors are drawn
   by original row index and the Ritz vectors come back in original order,
   so only rounding differs.  The relabelled copy lives in the workspace. */
#define LZ_REORDER_OFF 0       /* solve in the caller's order */
#define LZ_REORDER_HUBS 1      /* always relabel hub-first */
#define LZ_REORDER_AUTO 2      /* relabel when n >= 2^17 and the longest row
                                  holds at least 32 times the mean row
                                  length (power-law graphs); default */

/* Arithmetic of the FP32 storage mode (Sec. III-A keeps the intermediate
   operations of every kernel in double while vectors are stored in float;
   Sec. IV-D compares that with all-double and all-float runs).  Jacobi, the
   Ritz vectors and the report are FP64 in every mode. */
#define LZ_ARITH_MIXED 0       /* dots, norms and reorthogonalisation in FP64,
                                  SpMV accumulation in the storage's working
                                  precision; default */
#define LZ_ARITH_FP32 1        /* all-float: dots, norms, reorthogonalisation,
                                  the Gram correction, alpha, beta and the SpMV
                                  epilogue in FP32 (the start vector's norm is
                                  summed in FP64, its scale rounded to FP32);
                                  LZ_FP32 storage only, else
                                  LZ_ERR_INVALID_ARG */

typedef struct lz_options {
    uint64_t seed;           /* start vector: u_r = U01(SplitMix64(seed, r)),
                                v_1 = u/||u||; default 0 */
    int32_t reorth;          /* LZ_REORTH_*; default LZ_REORTH_TWICE */
    int32_t report;          /* 1 (default): residuals and orthogonality */
    void* workspace;         /* device memory of workspace_bytes, or NULL:
                                the library allocates for the call */
    size_t workspace_bytes;
    int32_t profile;         /* 1: time the phases with HIP events recorded
                                on `stream` (fills the t_* report fields) */
    int32_t reorder;         /* LZ_REORDER_*; default LZ_REORDER_AUTO */
    int32_t arith;           /* LZ_ARITH_*; default LZ_ARITH_MIXED */
    int32_t max_restarts;    /* lanczos_topk_async: breakdowns the enqueued
                                iterations can absorb, 0..LZ_MAX_RESTART_BUDGET;
                                -1 (default) = m.  Ignored by the blocking
                                calls, which enqueue more iterations after
                                reading the step count back. */
    int32_t sweep;           /* LZ_SWEEP_*: sweep-block layout of a relabelled
                                matrix; default LZ_SWEEP_AUTO */
} lz_options;

/* Sweep-block layout of the relabelled matrix for the Lanczos-step SpMV
 * (lz_report.spmv_layout = LZ_LAYOUT_SWEEP): the rows are cut into blocks of
 * at most 4096 rows and 2^18 entries (FP64; 2048 and 2^17 in FP32 and BF16),
 * each block's entries are stored in
 * column order with their row inside the block, and one wavefront walks a
 * block gathering x in address order while it adds the products into per-row
 * sums in LDS.  Costs a segmented sort at setup and 10 (FP32), 14 (FP64) or
 * 8 (BF16) more bytes of workspace per entry, plus 8 bytes per entry of setup
 * scratch; needs nnz < 2^32.  AUTO takes it for n >= 2^22 when x (n entries
 * of the storage precision) is at least 64 MiB; ON whenever the matrix is
 * relabelled; OFF never.  lanczos_topk_workspace_size() reports the AUTO
 * size; lanczos_topk_workspace_size_opt() the size for given options. */
#define LZ_SWEEP_AUTO (-1)
#define LZ_SWEEP_OFF 0
#define LZ_SWEEP_ON 1

#define LZ_MAX_RESTART_BUDGET 128

/* Matrix layouts of the Lanczos-step SpMV (lz_report.spmv_layout). */
#define LZ_LAYOUT_ROWS 0          /* caller's rows, entries in row order */
#define LZ_LAYOUT_RELABELLED 1    /* hub-first rows, entries in row order */
#define LZ_LAYOUT_TILE_SORTED 2   /* hub-first rows, each SpMV tile's entries
                                     in column order (2^20 < n < 2^22) */
#define LZ_LAYOUT_GROUP_SORTED 3  /* hub-first rows, entries of four
                                     consecutive tiles in column order
                                     (n <= 2^20) */
#define LZ_LAYOUT_SWEEP 4         /* hub-first rows in sweep blocks, each
                                     block's entries in column order
                                     (LZ_SWEEP_*) */
#define LZ_LAYOUT_XCACHE 16       /* flag: head of x staged in LDS */

/* Results of one solve: filled on the host when a blocking call returns, or
 * written to device memory by the last kernel of lanczos_topk_async. */
typedef struct lz_report {
    int32_t status;          /* lz_status of the solve */
    int32_t m_eff;           /* Lanczos steps taken (= m on success) */
    int32_t restarts;        /* breakdowns met: beta_{i+1} <= 100 u_w
                                max_j(|alpha_j| + beta_j), u_w the unit
                                roundoff of the working vector (2^-53 in
                                FP64 mode, 2^-24 in the FP32/BF16 modes) */
    int32_t jacobi_sweeps;
    double beta_last;        /* beta_{m+1}: norm of the final residual vector */
    double resid[LZ_MAX_STEPS];      /* ||A y_k - theta_k y_k|| / |theta_k|
                                        (= the absolute value if theta_k = 0) */
    double abs_resid[LZ_MAX_STEPS];  /* ||A y_k - theta_k y_k|| (Sec. IV-D) */
    double ortho_loss;       /* max |V^T V - I| over the m basis vectors */
    double ritz_ortho_loss;  /* max |Y^T Y - I| over the K Ritz vectors */
    double mean_angle_deg;   /* mean angle between Ritz vector pairs
                                (Sec. IV-D; 90 is ideal) */
    double alpha[LZ_MAX_STEPS];      /* diagonal of T */
    double beta[LZ_MAX_STEPS + 1];   /* beta[0] = 0, beta[i] couples v_i and
                                        v_{i+1} (1-based), beta[m] = beta_last */
    double theta[LZ_MAX_STEPS];      /* all m Ritz values (Jacobi order) */
    /* Phase timings in milliseconds (only with lz_options.profile = 1). */
    double t_setup_ms;       /* input checks, relabelling, tiles, start vector */
    double t_lanczos_ms;     /* all Lanczos iterations */
    double t_spmv_ms;        /* mean duration of one SpMV launch (the SpMV
                                of every eighth step is timed) */
    double t_orth_ms;        /* t_lanczos_ms / steps - t_spmv_ms: the rest of
                                a step (reorthogonalisation, launch gaps) */
    double t_finish_ms;      /* Jacobi, selection, Ritz vectors, report */
    int32_t reordered;       /* 1: the solve ran on the hub-first relabelling */
    int32_t spmv_layout;     /* matrix layout the Lanczos-step SpMV read:
                                LZ_LAYOUT_* plus LZ_LAYOUT_XCACHE when its
                                workgroups kept the head of x in LDS */
    int64_t bytes_streamed;  /* lanczos_topk_host: host-to-device bytes of
                                matrix entries (column indices and values)
                                copied during the solve, the one copy of the
                                resident slabs included; 0 otherwise */
} lz_report;

/* Fills *opt with the defaults above. */
void lz_options_init(lz_options* opt);

/* Human-readable name of a status code (static string). */
const char* lz_status_string(int status);

/*
 * Top-K eigenpairs of the symmetric CSR matrix (Sec. III, Algorithm 1 then
 * Jacobi and the Ritz product), the K eigenvalues of largest modulus.
 *   out_vals: device double[K], ordered by |lambda| descending, ties by
 *             lambda descending.
 *   out_vecs: device double[n*K], column-major (vector k at out_vecs+k*n),
 *             unit 2-norm, signed so its entry of largest modulus is positive.
 * Default options; the library allocates its workspace for the call
 * (stream-ordered, hipMallocAsync on `stream`).
 * Blocking: reads nnz = rowptr[n] and, after the m iterations, the step count
 * back from the device (more iterations follow breakdowns), and returns
 * after the results are in out_vals/out_vecs.  lanczos_topk_async is the
 * stream-ordered form.
 */
int lanczos_topk(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val,
                 int64_t n, int32_t K, int32_t m, int32_t precision, void* stream,
                 double* out_vals, double* out_vecs);

/* Device bytes of workspace a solve of this shape needs (default options). */
size_t lanczos_topk_workspace_size(int64_t n, int64_t nnz, int32_t K, int32_t m,
                                   int32_t precision);

/* The same for the given options (opt NULL: defaults): the sweep-block copy
 * (opt->sweep; none with opt->reorder = LZ_REORDER_OFF) changes it.  Returns 0
 * for invalid arguments or options.  Host-only, no device calls beyond
 * looking up the current device's properties. */
size_t lanczos_topk_workspace_size_opt(int64_t n, int64_t nnz, int32_t K, int32_t m,
                                       int32_t precision, const lz_options* opt);

/*
 * lanczos_topk with options and a report.  nnz must equal rowptr[n].
 * opt may be NULL (defaults); report may be NULL.  With a caller workspace
 * the call allocates nothing; otherwise the workspace is allocated and freed
 * stream-ordered on `stream`.  Blocking like lanczos_topk: it waits for the
 * device after the m iterations (breakdown check, and the choice of SpMV
 * variant once the row order is known) and at the end (report).
 */
int lanczos_topk_ex(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val,
                    int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t precision,
                    void* stream, double* out_vals, double* out_vecs,
                    const lz_options* opt, lz_report* report);

/*
 * Stream-ordered lanczos_topk_ex: every step is enqueued on `stream` and the
 * call returns without waiting for the device, so it can be pipelined with
 * other work or captured in a hipGraph (with a caller workspace: a
 * stream-ordered allocation inside a capture becomes a graph node).
 *   - The iterations are enqueued up front: m, plus opt->max_restarts more
 *     (default m) that absorb breakdowns (each restart takes one iteration
 *     that does not advance the step); those past the m-th step return at
 *     once.  A solve needing more ends with status LZ_ERR_RESTART_BUDGET in
 *     the report and leaves out_vals/out_vecs unwritten.
 *   - The hub-first relabelling is decided on the device; where the choice
 *     of SpMV variant depends on it, both variants are enqueued and the one
 *     that does not apply returns at once.
 *   - d_report: DEVICE pointer to an lz_report (or NULL), written by the last
 *     kernel; timings are zero, and numerical outcomes (breakdown budget,
 *     non-finite values, Jacobi limit, invalid column indices) appear only in
 *     its status.
 *   - Without opt->workspace the workspace is allocated with hipMallocAsync
 *     and freed with hipFreeAsync on `stream`.
 *   - opt->profile must be 0.
 * Argument errors are returned before anything is enqueued.  Results equal
 * those of lanczos_topk_ex with the same options bit for bit.
 */
int lanczos_topk_async(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val,
                       int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t precision,
                       void* stream, double* out_vals, double* out_vecs,
                       const lz_options* opt, lz_report* d_report);

/*
 * For callers that cannot allocate device memory (code under hipGraph
 * capture, tight serving loops, harnesses that forbid allocation):
 * lanczos_topk_async with its workspace in a fixed device array of the
 * library instead of opt->workspace or a stream-ordered allocation.  Same
 * arguments, kernels, results and report as lanczos_topk_async; the call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 *   - The array holds LZ_NOALLOC_SCRATCH_BYTES; a solve whose workspace
 *     (lanczos_topk_workspace_size) is larger returns LZ_ERR_TOO_LARGE.
 *   - opt->workspace must be NULL (else LZ_ERR_INVALID_ARG).
 *   - Every GPU the library runs on holds its own copy of the array until
 *     the process ends.  All calls on one GPU share it: calls that overlap
 *     on one GPU (other streams, other threads) race; order them on one
 *     stream.
 *   - The array's device address is looked up once per device, on the
 *     device's first call (that call returns LZ_ERR_HIP if it fails).
 */
#define LZ_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int lanczos_topk_noalloc(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val,
                         int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t precision,
                         void* stream, double* out_vals, double* out_vecs,
                         const lz_options* opt, lz_report* d_report);
/* LZ_NOALLOC_SCRATCH_BYTES, as the library was built. */
size_t lanczos_topk_noalloc_max_bytes(void);

/*
 * Host utility for tests and callers that want to check the symmetry the
 * solver assumes: returns 1 if the CSR matrix (host arrays; values in the
 * storage type of `precision`; duplicate entries summed) equals its
 * transpose, every pair of mirrored values agreeing within
 * rtol * max(|a_ij|, |a_ji|); 0 if not, with *bad_row (if non-NULL) set to a
 * row where it fails; a negative lz_status on invalid arguments (including
 * column indices outside [0, n)).
 */
int lz_check_symmetric(const int64_t* rowptr, const int32_t* col, const void* val, int64_t n,
                       int32_t precision, double rtol, int64_t* bad_row);

/*
 * lanczos_topk_ex on a matrix whose entries stay in host memory, for matrices
 * larger than device memory (the paper's out-of-core matrices: Sec. III-B
 * runs them through unified memory, Sec. IV-B measures them).
 *   host_rowptr: host int64[n+1] (any host memory); nnz = host_rowptr[n].
 *                Copied to the device once (8(n+1) bytes).
 *   host_col, host_val: host arrays of nnz entries in PINNED memory
 *                (hipHostMalloc or an equivalent page-locked allocation;
 *                anything else returns LZ_ERR_INVALID_ARG).  They are read
 *                by DMA while kernels run and must not change until the
 *                call returns.
 *   slab_nnz:    entries per streamed slab; 0 selects
 *                LZ_HOST_SLAB_NNZ_DEFAULT.  Slabs are runs of whole SpMV
 *                tiles of at most slab_nnz entries; two staging buffers of
 *                that size are allocated.  Must be >= 2048 and leave at most
 *                LZ_HOST_MAX_SLABS slabs.
 *   resident_nnz: leading entries (whole slabs) that stay on the device
 *                after one copy; 0 streams every slab at every pass,
 *                >= nnz keeps the whole matrix resident.
 * Every SpMV, and the residual product of the report, streams the
 * non-resident slabs from host memory on a copy stream of the call's own,
 * overlapped with the kernels of earlier slabs.  Column indices are checked
 * on the device in the first pass, before any kernel gathers through them.
 * The solve runs in the caller's row order: opt->reorder = LZ_REORDER_HUBS
 * returns LZ_ERR_INVALID_ARG and LZ_REORDER_AUTO does not relabel.  Results
 * equal lanczos_topk_ex with LZ_REORDER_OFF bit for bit in the modes whose
 * alpha comes from the orthogonalisation (LZ_REORTH_TWICE, _SELECTIVE);
 * with LZ_REORTH_NONE and _ONCE the alpha partial sums are grouped by slab.
 * opt->workspace (lanczos_topk_host_workspace_size bytes) covers the solve
 * state; the staging and resident buffers are allocated by the call and
 * freed before it returns.  report->bytes_streamed counts the copies.
 * Blocking.
 */
#define LZ_HOST_SLAB_NNZ_DEFAULT (int64_t)(1 << 24)
#define LZ_HOST_MAX_SLABS 16384
int lanczos_topk_host(const int64_t* host_rowptr, const int32_t* host_col, const void* host_val,
                      int64_t n, int32_t K, int32_t m, int32_t precision, int64_t slab_nnz,
                      int64_t resident_nnz, void* stream, double* out_vals, double* out_vecs,
                      const lz_options* opt, lz_report* report);

/* Device bytes of the workspace of lanczos_topk_host (no relabelled copy). */
size_t lanczos_topk_host_workspace_size(int64_t n, int64_t nnz, int32_t K, int32_t m,
                                        int32_t precision);

/*
 * y = A x in the given precision (Algorithm 1, the SpMV line), with the
 * same row partitioning and kernels the solver uses.  x and y are device
 * arrays of n elements of the storage type (y is double for LZ_FP64, float
 * otherwise).  The library allocates its scratch for the call.  Blocking.
 */
int lz_spmv(const int64_t* csr_rowptr, const int32_t* csr_col, const void* csr_val,
            int64_t n, int64_t nnz, int32_t precision, const void* x, void* y, void* stream);

/*
 * Eigen-decomposition of one symmetric tridiagonal matrix by the parallel
 * Jacobi kernel the solver uses (Sec. III, second phase).  Host arrays:
 * alpha[m] diagonal, offdiag[m-1]; out theta[m] (unsorted, Jacobi order),
 * S[m*m] row-major, column k = eigenvector of theta[k].  m <= LZ_MAX_STEPS.
 * Returns LZ_ERR_NOT_CONVERGED if the sweep limit was hit.  Blocking.
 */
int lz_tridiag_eig(const double* alpha, const double* offdiag, int32_t m,
                   double* theta, double* S, int32_t* sweeps);

/*
 * Orthogonality loss max_{i,j} |(X^T X - I)_{ij}| of c <= LZ_MAX_STEPS
 * columns of a column-major device matrix X (leading dimension ldx >= n,
 * storage type of `precision`), computed by the Gram kernel of the solve
 * report (Sec. IV-D: orthogonality of the computed vectors).  Blocking.
 */
int lz_ortho_loss(const void* X, int64_t ldx, int64_t n, int32_t c, int32_t precision, void* stream,
                  double* out_loss);

/* ------------------------------------------------------------------ */
/* Serving: a request loop that admits Top-K solves as they arrive, keeps
 * each admitted request's CSR and Lanczos state resident in a fixed HBM
 * arena, and runs admitted requests concurrently on their own HIP streams
 * (continuous batching).  A request is admitted when a slot is free and its
 * footprint (CSR + workspace + outputs) fits in the arena; the queue is FIFO
 * with bounded backfill.  Results do not depend on what else is running:
 * every kernel's launch shape depends only on the request itself.  All
 * pointers in lz_request are HOST pointers owned by the caller and must stay
 * valid until the request has completed (pinned memory copies faster). */
typedef struct lz_server lz_server;

typedef struct lz_request {
    const int64_t* rowptr;   /* host int64[n+1] */
    const int32_t* col;      /* host int32[nnz] */
    const void* val;         /* host values in the storage precision */
    int64_t n, nnz;
    int32_t K, m, precision, reorth;   /* reorth: LZ_REORTH_* */
    uint64_t seed;
    double* out_vals;        /* host double[K], written on completion */
    double* out_vecs;        /* host double[n*K] column-major, or NULL */
    double* out_resid;       /* host double[K]: relative residual of each
                                returned pair (Top-K order, as out_vals),
                                written on completion; or NULL */
} lz_request;

typedef struct lz_result {
    int32_t status;          /* lz_status of the solve */
    int32_t m_eff, restarts, slot;
    double t_submit_ms;      /* host steady clock, ms since server creation */
    double t_admit_ms;
    double t_done_ms;        /* when the server observed completion */
    double device_ms;        /* first copy to last kernel, on the device */
    double resid_max;        /* max relative residual over the K pairs */
    double ortho_loss;       /* max |V^T V - I| of the basis */
} lz_result;

typedef struct lz_server_stats {
    uint64_t submitted, completed, rejected, active, queued;
    size_t arena_bytes, arena_in_use, arena_peak;
    double worker_enqueue_ms;  /* host time the slot worker threads spent
                                  enqueueing work (copies, graph capture and
                                  launch, finish, completion) since the server
                                  started, summed over the threads (so it can
                                  exceed the wall time) */
} lz_server_stats;

/* Creates a server on `device` with an HBM arena of hbm_budget_bytes and at
 * most max_slots requests in flight; use_graphs = 1 captures each request's
 * Lanczos iterations in a hipGraph.  Each slot gets its own stream and its
 * own host worker thread.  LZ_ERR_OUT_OF_MEMORY if the arena, or a worker
 * thread, cannot be had; LZ_ERR_HIP if a stream, an event or pinned state
 * cannot be created. */
int lz_server_create(int device, size_t hbm_budget_bytes, int32_t max_slots, int32_t use_graphs,
                     lz_server** out);

/* Device bytes a request occupies while admitted (0 for invalid shapes). */
size_t lz_request_footprint(int64_t n, int64_t nnz, int32_t K, int32_t m, int32_t precision);

/* Queues a request; returns LZ_ERR_TOO_LARGE if it can never fit. */
int lz_server_submit(lz_server* s, const lz_request* req, uint64_t* ticket);

/* LZ_PENDING while the request runs; otherwise its final status, with *res
 * filled (res may be NULL).  A finished ticket can be polled again. */
int lz_server_poll(lz_server* s, uint64_t ticket, lz_result* res);

/* Blocks until the request has finished; returns its status. */
int lz_server_wait(lz_server* s, uint64_t ticket, lz_result* res);

int lz_server_get_stats(lz_server* s, lz_server_stats* out);

/* Waits for every queued and running request, stops the slot worker
 * threads and frees the arena. */
int lz_server_destroy(lz_server* s);

#ifdef __cplusplus
}
#endif

#endif /* LANCZOS_TOPK_H */
