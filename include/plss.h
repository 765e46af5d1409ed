/* plss.h -- C ABI of the PLSS GPU library (AMD MI355X, gfx950).
 *
 * PLSS (Brust & Saunders, "PLSS: A Projected Linear Systems Solver",
 * arXiv:2207.07615) solves a consistent system A x = b, A (m x n) sparse,
 * b in range(A) (Section 1, eq. axb), by x_k = x_{k-1} + p_k (eq. xko) where
 * p_k is the minimum-norm correction satisfying the sketched constraints
 * S_kᵀ A (x_{k-1} + p_k) = S_kᵀ b (eqs. itProb-cons, closed form eq. pkLong).
 *
 *  - Residual sketch S_k = [r_0 ... r_{k-1}] (eq. S): the short recurrence of
 *    Theorem 2 / Algorithm 1 (one product with A and one with Aᵀ per
 *    iteration, four vectors).
 *  - Identity sketch S_k = [e_{i_1} ... e_{i_k}] (Section 7, eq. pkKacz,
 *    "PLSS Kaczmarz"), with the stored products A p_j.
 *  - Mixed sketch: residual and identity columns alternate, one row per
 *    residual column (a sketch of the general form of Section 2).
 *
 * Conventions for every call:
 *  - Return value: plss_status.  0 = success; > 0 = finished with a warning
 *    (outputs valid); < 0 = error (outputs unspecified).  On error,
 *    plss_last_error() returns a description (thread-local).
 *  - Array arguments may point to host memory or to device memory of the
 *    handle's GPU (unified addressing; the library copies what it needs).
 *    They are read (or written, for outputs) only during the call.
 *  - Handles, matrices and servers are owned by the library until their
 *    *_destroy call.  One handle per host thread; calls on one handle are
 *    serialised on the handle's HIP stream and return when their work is
 *    complete.
 */
#ifndef PLSS_H
#define PLSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PLSS_OK = 0,             /* stop test met */
  PLSS_NOT_CONVERGED = 1,  /* iteration limit reached; x is the last iterate */
  PLSS_BREAKDOWN = 2,      /* phi == 0 or sqrt(theta*phi)/rho <= 1 (b not in range(A)
                              in exact arithmetic); x is the last iterate */
  PLSS_PENDING = 3,        /* server: request not finished yet */
  PLSS_EINVAL = -1,        /* malformed argument (CSR, sizes, tolerances, NaN, permutation) */
  PLSS_ENOMEM = -2,        /* device allocation failed or over the memory budget */
  PLSS_EDEVICE = -3,       /* HIP runtime error */
  PLSS_ECANCELLED = -4     /* server: request cancelled */
} plss_status;

typedef enum {
  PLSS_SKETCH_RESIDUAL = 0, /* eq. S, Algorithm 1 */
  PLSS_SKETCH_IDENTITY = 1, /* Section 7 (PLSS KZ) */
  PLSS_SKETCH_MIXED = 2,    /* r_{k-1}, e_{i}, r, e, ... alternating */
  PLSS_SKETCH_BLOCK_IDENTITY = 3, /* opts.block identity columns appended per step: the
                                     block form of the triangular update of Section 2.4 */
  PLSS_SKETCH_BLOCK_MIXED = 4,    /* r_{k-1} and opts.block identity columns per step */
  PLSS_SKETCH_RANDPROJ = 5        /* Section 8's randomized projection: eq. pkLong with a
                                     fresh m x opts.block standard normal sketch per step */
} plss_sketch;

typedef enum {
  PLSS_F64 = 0, /* values stored and streamed in float64 */
  PLSS_F32 = 1  /* values stored in float32 (rounded to nearest); products
                   accumulate in float32; dots, norms, scalars, x and the
                   refinement residual stay in float64 */
} plss_dtype;

/* A sparse matrix in CSR form, as given by the caller.  row_ptr has m+1
 * non-decreasing entries with row_ptr[0] = 0 and row_ptr[m] = nnz; the
 * column indices of a row are ascending, distinct and in [0, n); values
 * are finite float64. */
typedef struct {
  int64_t m, n, nnz;
  const int64_t* row_ptr;
  const int32_t* col_idx;
  const double* values;
} plss_csr;

typedef struct {
  plss_sketch sketch;
  double tol;           /* stop when ||r|| <= tol*||b|| (or <= tol if tol_absolute);
                           the stop rule stated after Algorithm 1 */
  int64_t maxit;        /* at most maxit updates (Algorithm 1's maxIt > 0) */
  int32_t tol_absolute;
  int32_t refine;       /* float32 storage: float64 iterative refinement on b - A x */
  double inner_tol;     /* refinement: relative tolerance of each inner solve */
  int64_t max_outer;    /* refinement: bound on inner solves */
  const double* x0;     /* optional start (length n); NULL means x0 = 0 */
  const double* wi_diag;/* optional diagonal of BᵀB (length n, > 0): W = diag(1/wi)
                           (Section 4.1); NULL means W = I.  Residual sketch only. */
  const int32_t* row_perm; /* identity/mixed: order of identity columns, a permutation
                              of 0..m-1 reused cyclically; NULL means 0..m-1 */
  int64_t hist_cap;     /* identity/mixed/block: history columns kept before the
                           stored history is cleared (0: min(m, n, 256); at most
                           256 for identity/mixed, 1024 for the block sketches) */
  int32_t chunk;        /* iterations per launch batch between host checks (0: auto;
                           the residual sketch predicts it from the observed
                           decrease of the residual, and takes at most 256) */
  int32_t timing;       /* record per-kernel device times with events around the
                           phases of one iteration in eight (see plss_kernel_times) */
  int32_t engine;       /* residual sketch: 0 = automatic, 1 = one launch per phase
                           (all CUs on the system), 2 = single workgroup: the whole
                           solve in one workgroup, vectors and row pointers in
                           LDS (requires 8n + (m + 2n) x vector bytes +
                           4 (m + n) <= 156 KiB, about m + 3.5 n <= 19,900 in
                           float64; automatic for those systems with at most 2^18
                           entries) */
  int32_t block;        /* block sketches: identity rows per step (1..16 identity,
                           1..15 mixed); randomized projection: sketch columns
                           (1..16) */
  uint64_t seed;        /* randomized projection: Philox4x32-10 key (low word, high
                           word); entry [i, 4q + t] of the k-th sketch is normal t
                           (Box-Muller) of the counter (i, k, q, 0) */
} plss_opts;

typedef struct {
  int64_t iters;        /* updates applied (summed over inner solves) */
  int64_t outer_iters;  /* inner solves (1 without refinement) */
  double relres;        /* last recursive residual estimate / ||b|| */
  double relres_true;   /* ||b - A x|| / ||b|| computed in float64 at exit */
  int32_t status;       /* plss_status of this system */
  double ms;            /* device time of the solve (milliseconds) */
} plss_info;

typedef struct plss_handle plss_handle;
typedef struct plss_matrix plss_matrix;
typedef struct plss_server plss_server;

/* Fill opts with defaults: residual sketch, tol 1e-8 relative, maxit 1000,
 * refine on, inner_tol 1e-4, max_outer 20, everything else 0/NULL. */
void plss_opts_default(plss_opts* opts);

/* Create a handle on GPU `device` (its own non-blocking stream).  The calls
 * on a handle are serialised and keep their device scratch on it between
 * calls, growing it as needed and never shrinking it: launch tables,
 * per-system scalars and vectors, a pinned state mirror; for the multi-RHS
 * solves their dense blocks; for the identity and mixed sketches a history block of
 * about 8 (m + n) hist_cap bytes; for the block sketches about
 * 8 (m + n) hist_cap bytes too (hist_cap up to 1024); for the randomized
 * projection 8 (m + n) r bytes (r rounded up to 4).  The largest such block a
 * handle has needed stays allocated until plss_release_workspace or
 * plss_destroy (a server created on the handle does not count it in its HBM
 * budget; use a separate handle for sketch solves beside a server with a
 * tight budget, or release the workspace after them). */
plss_status plss_create(plss_handle** h, int device);
plss_status plss_destroy(plss_handle* h);
/* Free the handle's scratch described above (device blocks, pinned mirror,
 * launch lists, events and second stream) after its pending work; the next
 * call on the handle allocates afresh.  Matrices, servers and results are
 * untouched, and results do not depend on it.  Errors: EINVAL for a null
 * handle. */
plss_status plss_release_workspace(plss_handle* h);

/* Upload A and build its device store once: CSR with int32 pointers and the
 * CSC copy (rows ascending inside every column) used for the products with
 * Aᵀ (Algorithm 1's y = Aᵀ r), values in `storage` precision, and the tile
 * tables of both.  The first identity or mixed sketch solve on a matrix whose
 * n float64 entries exceed 3 MB adds a copy of A split into 8 column blocks
 * (one per XCD, equal entry counts) for its products A p; it stays with the
 * matrix (plss_matrix_info counts it).  Errors: EINVAL for a malformed CSR or
 * nnz >= 2^31, ENOMEM. */
plss_status plss_matrix_create(plss_handle* h, const plss_csr* A, plss_dtype storage,
                               plss_matrix** out);
plss_status plss_matrix_destroy(plss_matrix* A);
/* Sizes and device bytes held by the store. */
plss_status plss_matrix_info(const plss_matrix* A, int64_t* m, int64_t* n, int64_t* nnz,
                             int64_t* device_bytes);
/* Copy the CSC copy out: col_ptr (n+1, int64), row_idx (nnz), values (nnz, float64,
 * widened from the storage precision).  Any pointer may be NULL. */
plss_status plss_matrix_csc(const plss_matrix* A, int64_t* col_ptr, int32_t* row_idx,
                            double* values);
/* Re-tile both directions for the tile width (entries per thread, 4, 8 or
 * 16) that runs fastest on this device; returns the widths chosen. */
plss_status plss_matrix_autotune(plss_handle* h, plss_matrix* A, int32_t* csr_width,
                                 int32_t* csc_width);

/* Layout of the two products of every residual-sketch iteration
 * (Algorithm 1: the residual update with A p and y = Aᵀ r).
 *  - Tiles (0): the CSR / CSC tile tables; every product gathers its input
 *    vector from memory.
 *  - Stripes (1): a striped copy of the direction.  One workgroup owns a unit
 *    of rows and keeps their sums in LDS while the input vector passes
 *    through LDS in stripes; the entries of a unit are stored stripe by
 *    stripe.  Products with A: units of at most 8192 rows, stripes of 6144
 *    entries.  For Aᵀ the rows of A are first split into 8 blocks (one per
 *    XCD) and each block gets its own striped store (units of at most 16384
 *    rows, stripes of 2048 entries); the block products are summed in block
 *    order.
 * Both layouts give deterministic sums (a fixed order per matrix) and the
 * same results up to rounding.  plss_matrix_create picks stripes for a
 * direction when the matrix has at least 2^23 entries and every unit reading
 * its slice of the input vector costs less than the entries streamed. */
typedef struct {
  int32_t a_stripes;    /* products with A use the striped store */
  int32_t t_stripes;    /* products with Aᵀ use the striped row-block stores */
  int32_t unit_rows;    /* rows per unit, 1..16384 (at most 8192 are used for A);
                           0 = chosen from the shape, and for A the unit
                           boundaries then moved so that the units hold about
                           equal entry counts (as many units as at the chosen
                           row count, at most 8192 rows each); reads back as
                           that row count */
} plss_layout;
/* Read (got) and / or change (want) the layout of A; want = NULL only reads.
 * Building a striped store takes about (4 + value bytes) per entry of device
 * memory per direction and a few milliseconds per 10^8 entries; dropping one
 * frees it.  plss_spmv and the residual-sketch solves use the layout in
 * force at the time of the call (the identity and mixed sketches always use
 * the tiles).  Errors: EINVAL for unit_rows outside [0, 16384] or more than
 * 8192 stripes (n above 50.3 million or m/8 above 16.7 million), ENOMEM; on error the
 * directions whose store could not be built fall back to tiles. */
plss_status plss_matrix_layout(plss_handle* h, plss_matrix* A, const plss_layout* want, plss_layout* got);

/* y = A x (transpose = 0, x length n, y length m) or y = Aᵀ x (transpose = 1),
 * float64 in and out, float64 accumulation over the stored values. */
plss_status plss_spmv(plss_handle* h, const plss_matrix* A, int transpose, const double* x,
                      double* y);

/* Bytes of the fixed device array behind plss_spmv_noalloc: one per GPU the
 * library runs on, held from the library's load until the process ends. */
#define PLSS_NOALLOC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP stream
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as plss_spmv, computed by the same kernels (bit-identical results),
 * with no hipMalloc, hipFree or host-pinned allocation.  x (length n, or m
 * for transpose = 1) and y (length m, or n) must be device memory of the
 * handle's GPU and must not overlap; the caller owns both.  The scratch of
 * the product (launch descriptor, launch list and, for the striped
 * transposed product, the per-row-block partial vectors: 8 * row blocks * n
 * bytes) lives in that GPU's fixed array of PLSS_NOALLOC_SCRATCH_BYTES; its
 * device address is looked up once per GPU at plss_create.  The array keeps
 * the last call's contents; nothing in it needs to start at zero.  Calls in
 * one process that use the same GPU share the array and are serialised by a
 * lock (overlapping calls would race on it); returns when y is complete.
 * Errors: EINVAL for host or foreign-device pointers, overlapping x and y,
 * or a product whose scratch exceeds the array (the message gives both
 * sizes); EDEVICE if the array's address cannot be found. */
plss_status plss_spmv_noalloc(plss_handle* h, const plss_matrix* A, int transpose, const double* x,
                              double* y);

/* Both matrix products of one residual-sketch iteration (Algorithm 1,
 * Section 5: the residual update with A p, then y = Aᵀ r with the updated
 * residual) in one pass over the CSR store of A, as an alternative to the
 * second pass over the transposed store:
 *   r (length m, in/out): r <- r - A p;
 *   y (length n, out):    y = Aᵀ r, with the updated r;
 *   rho_phi (host, 2 doubles, may be NULL): ||r||² and ||y||² after the call.
 * Level 1 streams the rows once: row i's dot product, the update of r_i, and
 * the row's contributions a_ij r_i.  Level 2 sums column j's contributions
 * in ascending row order.  Every sum has a fixed order, so results are
 * bit-reproducible; float64 arithmetic over the stored (float64 or float32)
 * values.  The first call on a matrix builds its map from transposed
 * positions to row positions and a contribution buffer (4 + 8 bytes per
 * entry), kept with the matrix until plss_matrix_destroy.  p, r and y may be
 * host or device memory (device memory of the handle's GPU is used in
 * place, otherwise the vectors are staged through the handle's workspace) and
 * must not overlap.  Returns when r, y and rho_phi are complete.  Errors:
 * EINVAL for null arguments, ENOMEM. */
plss_status plss_residual_pair(plss_handle* h, plss_matrix* A, const double* p, double* r, double* y,
                               double* rho_phi);

/* Solve A x = b (b length m, x length n).  res_hist (may be NULL) receives
 * up to hist_cap entries sqrt(rho_k)/||b||, k = 0..iters (the recursive
 * residual of Algorithm 1).  Returns the system's status (OK, NOT_CONVERGED,
 * BREAKDOWN) or an error. */
plss_status plss_solve(plss_handle* h, const plss_matrix* A, const double* b,
                       const plss_opts* opts, double* x, double* res_hist, int64_t hist_cap,
                       plss_info* info);

/* Solve nsys independent systems together: every phase of an iteration is
 * one launch over all unfinished systems.  Each result equals the result of
 * solving that system alone with plss_solve (the reductions of a system
 * depend only on its own tiles).  opts, b, x and info are arrays of nsys.
 * Returns PLSS_OK if every system converged, else the first non-OK status. */
plss_status plss_solve_batch(plss_handle* h, int32_t nsys, const plss_matrix* const* A,
                             const double* const* b, const plss_opts* opts, double* const* x,
                             plss_info* info);

/* Solve A X = B for nrhs right-hand sides (B m x nrhs and X n x nrhs, both
 * column-major): nrhs independent residual-sketch recurrences whose
 * products with A and Aᵀ are one sparse x dense block product each.
 * info: array of nrhs.  Residual sketch only. */
plss_status plss_solve_multi(plss_handle* h, const plss_matrix* A, int32_t nrhs, const double* B,
                             const plss_opts* opts, double* X, plss_info* info);

/* Per-kernel device time accumulated while opts.timing was set, and the
 * number of launches: index 0 = product with A (r <- r - A p), 1 = product
 * with Aᵀ (y <- Aᵀ r; with row blocks of Aᵀ, the block products), 2 = sum of
 * the block products (when there are row blocks) and step scalars, 3 =
 * vector update.  Resets the counters. */
plss_status plss_kernel_times(plss_handle* h, double* ms4, int64_t* launches4);

/* ---- request loop (continuous batching) ----
 * A server owns a host thread and its own streams on the handle's device.
 * Submitted systems wait until their device footprint fits under
 * hbm_budget_bytes and a slot is free, are uploaded and transposed on a side
 * stream, then join the running batch at the next launch boundary; all
 * admitted systems advance together on the per-phase engine (opts.engine 0
 * and 1 alike).  A request with opts.engine = 2 runs whole in one workgroup
 * on a stream of its own beside the batch.  Finished solutions are copied
 * back and their memory freed.  A served result equals the solve of the same
 * system alone on the same engine, bit for bit. */
plss_status plss_server_create(plss_handle* h, size_t hbm_budget_bytes, int32_t max_slots,
                               plss_server** out);
/* Queue a system (A is copied; the caller's arrays are free after return).
 * *req receives the request id.  EINVAL for malformed input, ENOMEM if the
 * system alone exceeds the budget. */
plss_status plss_server_submit(plss_server* s, const plss_csr* A, plss_dtype storage,
                               const double* b, const plss_opts* opts, uint64_t* req);
/* PLSS_PENDING while running; otherwise writes x (length n, host memory) and
 * info and releases the request (a second poll returns EINVAL). */
plss_status plss_server_poll(plss_server* s, uint64_t req, double* x, plss_info* info);
/* Block until every submitted request has finished. */
plss_status plss_server_drain(plss_server* s);
/* Cancel a queued or running request; its poll then returns ECANCELLED. */
plss_status plss_server_cancel(plss_server* s, uint64_t req);
/* Server counters: submitted, finished, admitted-now, peak bytes in use. */
plss_status plss_server_stats(plss_server* s, int64_t* submitted, int64_t* finished,
                              int64_t* active, int64_t* peak_bytes);
plss_status plss_server_destroy(plss_server* s);

const char* plss_status_string(plss_status s);
const char* plss_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PLSS_H */
