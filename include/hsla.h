/*
 * hsla -- differentiable sparse Krylov solves on one MI355X (gfx950).
 *
 * C ABI of libhsla.so.  Plain pointers and sizes only.  Every `d_*`
 * argument is a device pointer on the handle's device, owned by the caller
 * (the library never frees it and keeps no reference past the call unless
 * stated).  Host pointers are named without the prefix.  Device work is
 * ordered after everything already enqueued on the `stream` argument (a
 * hipStream_t passed as void*; NULL means the legacy default stream): the
 * library runs it on a private stream of default priority that waits on an
 * event recorded on `stream`, and every call returns only after its device
 * work has completed, so outputs are valid for later work on any stream.
 *
 * Errors: every entry point returns hsla_status.  0 = success; > 0 =
 * warning with valid output; < 0 = error, outputs undefined.  A message for
 * the last error on a handle is available from hsla_last_error().  No C++
 * exception crosses this boundary.  A handle is not thread-safe; patterns
 * may be shared by handles on one device and change only through
 * hsla_pattern_set_format.
 *
 * The problem statement is the paper's x = A.solve(b) with A given by a
 * sparsity pattern and values, differentiable in both the values and b
 * (arXiv 2601.13994, Sec. "API" and the API listing of the appendix).
 */
#ifndef HSLA_H
#define HSLA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hsla_status {
    HSLA_OK = 0,
    HSLA_NOT_CONVERGED = 1, /* max_iter reached; x holds the last iterate       */
    HSLA_BREAKDOWN = 2,     /* p^T A p <= 0 (CG) or a BiCGStab breakdown after
                               its one restart; x holds the last iterate.  Also
                               before the first iteration (x = x0) when Jacobi
                               meets a negative diagonal under CG, or an FSAI
                               factor holds a non-finite value or a row whose
                               last entry is not a positive diagonal          */
    HSLA_FELL_BACK = 3,     /* learned preconditioner rejected, Jacobi used     */
    HSLA_STAGNATED = 4,     /* stall_window set and ||r_k|| fell less than 10x
                               over the last stall_window iterations; x holds
                               the last iterate                                */
    HSLA_ERR_INVALID_ARG = -1,
    HSLA_ERR_INVALID_CSR = -2, /* pattern not canonical CSR (see hsla_pattern_create) */
    HSLA_ERR_NONFINITE = -3,   /* NaN/Inf met in b, values or a recurrence      */
    HSLA_ERR_HIP = -4,         /* HIP runtime error                              */
    HSLA_ERR_NO_MEMORY = -5,
    HSLA_ERR_ZERO_DIAGONAL = -6, /* Jacobi requested but a diagonal is missing or 0 */
    HSLA_ERR_INTERNAL = -7
} hsla_status;

/* CG_SR: CG with the single-reduction recurrence of Chronopoulos and Gear
 * (the same iterates in exact arithmetic, different rounding): w = A r, and
 * r.r and w.r in one reduction per iteration instead of two (the roadmap
 * after the paper's Algorithm "Distributed CG", appendix "Distributed
 * Conjugate Gradient and Halo Exchange").  It runs with no or Jacobi
 * preconditioning on the per-iteration kernels (three launches per
 * iteration instead of five; one more vector, s = A p, is streamed) and in
 * the persistent kernels, shared-pattern and ragged (one workgroup
 * reduction and two passes per iteration instead of two and three); FSAI
 * and the segmented ragged path run it as CG.  hsla_info.method reports
 * which ran.
 *
 * HSLA_METHOD_CG_SSTEP is s-step (communication-avoiding) CG, the other
 * roadmap item of that appendix, in Carson and Demmel's formulation of the
 * s-step method of Chronopoulos and Gear: per outer iteration 2s - 1 SpMVs
 * build the Chebyshev basis on [0, 2] of the Krylov spaces of p and r
 * (hsla_opts.s_step = s inner steps, 2..4), one pass forms their Gram
 * matrices (the only reduction of the outer iteration), the s CG steps run
 * on coordinate vectors, and one sweep recovers x, r and p.  In exact
 * arithmetic its iterates are CG's.  It runs on the Jacobi-scaled operator
 * (precond JACOBI only; other preconditioners are rejected), on the
 * per-iteration kernels (never in a persistent launch) and without
 * profiling; the stop test follows every inner step on the unscaled
 * residual from the weighted Gram matrix. */
typedef enum hsla_method {
    HSLA_METHOD_AUTO = 0,
    HSLA_METHOD_CG = 1,
    HSLA_METHOD_BICGSTAB = 2,
    HSLA_METHOD_CG_SR = 3,
    HSLA_METHOD_CG_SSTEP = 4
} hsla_method;
typedef enum hsla_precond { HSLA_PRECOND_NONE = 0, HSLA_PRECOND_JACOBI = 1, HSLA_PRECOND_FSAI = 2 } hsla_precond;

typedef struct hsla_handle hsla_handle;
typedef struct hsla_pattern hsla_pattern;

/* Solver options.  hsla_opts_default() fills the defaults noted here. */
typedef struct hsla_opts {
    int32_t method;      /* hsla_method; AUTO = CG if A equals A^T bit for bit, else BiCGStab */
    int32_t precond;     /* hsla_precond; default JACOBI                                        */
    double rtol;         /* stop when ||r_k||_2 <= max(rtol*||b||_2, atol); default 1e-8         */
    double atol;         /* default 0                                                           */
    int64_t max_iter;    /* <= 0: min(10 n, 100000)                                             */
    int32_t check_every; /* iterations between host convergence checks; <= 0: automatic          */
    int32_t use_x0;      /* 1: d_x holds the initial guess on input; default 0 (x0 = 0)          */
    int32_t use_graph;   /* 1: replay iteration chunks as HIP graphs; default 1                  */
    int32_t profile;     /* 1: time every SpMV(+dot) launch of the iteration with HIP events
                            (graphs off); results in hsla_info.spmv_ms / spmv_launches          */
    const float *d_G;    /* FSAI: G values on the lower pattern (float32, [B][nnz_L]); else NULL */
    const float *d_GT;   /* FSAI: the same values in G^T's CSR order ([B][nnz_L])               */
    int32_t persistent;  /* 1 (default): CG with Jacobi or no preconditioner (x0 = 0, profile off)
                            on systems of at most 4096 rows of <= 16 entries, or on batches of at
                            least one system per compute unit with at most 131072 entries each,
                            runs as one persistent launch, one workgroup per system;
                            0: always per-iteration kernels (ragged batches: the segmented path);
                            2: as 1, and ragged batches always run in one persistent launch     */
    int32_t stall_window;/* > 0: a system whose recursive ||r_k|| has not fallen by 10x within
                            stall_window iterations (counted from the start or from the last
                            iteration where it had) stops with HSLA_STAGNATED, e.g. so that a
                            poor learned preconditioner gives way to Jacobi early.  Runs on the
                            per-iteration kernels (no persistent launch).  Default 0: off     */
    int32_t s_step;      /* HSLA_METHOD_CG_SSTEP: inner steps per outer iteration, 2..4;
                            default 4                                                        */
} hsla_opts;

/* Per-system result information. */
typedef struct hsla_info {
    int64_t iters;        /* iterations run (one SpMV per CG iteration, two per BiCGStab)  */
    int32_t status;       /* hsla_status of this system                                    */
    int32_t method;       /* method actually used                                          */
    double rel_residual;  /* recursive ||r_k|| / ||b|| (||r_k|| if b = 0)                   */
    double true_residual; /* ||b - A x||_2 / ||b||_2 recomputed in FP64 at the end         */
    double spmv_ms;       /* profile mode: summed duration of the SpMV(+dot) launches that
                             did work (all systems of a batch share one launch)            */
    int64_t spmv_launches;/* profile mode: number of those launches                        */
    int32_t spmv_form;    /* SpMV form of the solve: 0 row tiles (CSR or row masks),
                             1 per-solve diagonal-major copy, 2 its symmetric half form
                             (main and upper diagonals stored), 3 one persistent launch,
                             4 the half form of Jacobi CG's scaled operator (upper
                             diagonals only; its diagonal is 1), 5 the full copy of
                             right-Jacobi BiCGStab's A D^{-1} without its unit diagonal    */
    int32_t spmv_paired;  /* 1 if the diagonal forms ran two adjacent rows per thread: 5, 7
                             or 9 diagonals with offsets -1, 0, +1 in the middle, every
                             other offset even and n even; that layout reads no row masks
                             (absent entries are stored as 0).  0 otherwise              */
    double t_start_ms;    /* persistent launches (spmv_form 3): when the workgroup that ran
                             this system began it and ended it, on the device clock, in ms
                             after the earliest start in the launch; 0 elsewhere          */
    double t_end_ms;
    int32_t workgroups;   /* persistent launches: workgroups the launch started; 0 elsewhere */
    int32_t reserved;
} hsla_info;

void hsla_opts_default(hsla_opts *opts);
const char *hsla_status_string(int status);

/* ---------------------------------------------------------------- handle */
/* Creates a handle bound to `device` (a HIP device ordinal).  The handle owns
 * its workspace (grown on demand, released by hsla_destroy). */
hsla_status hsla_create(hsla_handle **out, int device);
void hsla_destroy(hsla_handle *h);
const char *hsla_last_error(const hsla_handle *h);

/* Device memory of the handle's workspaces (solver vectors and partials,
 * per-solve diagonal-major copies, network activations, adjoint
 * temporaries).  By default the library calls hipMalloc/hipFree; with an
 * allocator set, it calls alloc(bytes, ctx) (which must return device memory
 * on the handle's device aligned to 256 bytes, or NULL) and free(ptr, ctx),
 * e.g. a framework's caching allocator.  Setting it releases the handle's
 * current workspaces first (after waiting for the device).  alloc and free
 * are both NULL (back to hipMalloc) or both set.  Pattern buffers are
 * allocated with hipMalloc at pattern creation. */
typedef void *(*hsla_alloc_fn)(size_t bytes, void *ctx);
typedef void (*hsla_free_fn)(void *ptr, void *ctx);
hsla_status hsla_set_allocator(hsla_handle *h, hsla_alloc_fn alloc, hsla_free_fn free, void *ctx);
/* Workspace bytes a solve of B systems on `p` with `opts` (NULL: defaults)
 * takes from the handle (AUTO method: the larger of CG and BiCGStab), and
 * hsla_reserve grows the workspace to at least `bytes` now, so that later
 * calls needing no more than that allocate nothing for it. */
hsla_status hsla_workspace_size(hsla_handle *h, const hsla_pattern *p, int32_t B, const hsla_opts *opts,
                                size_t *bytes);
hsla_status hsla_reserve(hsla_handle *h, size_t bytes);

/* --------------------------------------------------------------- pattern */
/* A sparsity pattern shared by one matrix or by a batch of value sets: the
 * paper's single-matrix sparse tensor, which holds one matrix or a batch
 * sharing one pattern so that the per-pattern work is done once (Sec.
 * "Unified Backend Abstraction", paragraph "Typed sparse-tensor hierarchy").
 * The paper stores COO with 64-bit indices; this library takes canonical CSR
 * with 32-bit indices.
 *
 * Validates and copies a CSR sparsity pattern (row_ptr int32[n+1], col
 * int32[nnz], device memory) and derives the per-pattern data every solve
 * reuses: diagonal positions, the transpose permutation, symmetry of the
 * pattern, the lower triangle, and the SpMV tile schedule.  Canonical CSR
 * means: 0-based, row_ptr[0] = 0, row_ptr nondecreasing, row_ptr[n] = nnz,
 * 0 <= col < n, columns strictly increasing within a row, nnz < 2^31.
 * Explicit zeros are legal; empty rows are legal for SpMV but a solve
 * rejects a missing diagonal under Jacobi.  Returns HSLA_ERR_INVALID_CSR
 * (with the first bad row in hsla_last_error) otherwise.  The caller's
 * buffers are not retained.  `flags` is 0 or HSLA_PATTERN_CSR (no
 * offset-mask forms are derived: the pattern behaves as after
 * hsla_pattern_set_format(p, HSLA_FORMAT_CSR) for good, and creation skips
 * their detection); other bits give HSLA_ERR_INVALID_ARG. */
enum { HSLA_PATTERN_CSR = 1u };
hsla_status hsla_pattern_create(hsla_handle *h, int32_t n, int64_t nnz, const int32_t *d_row_ptr,
                                const int32_t *d_col, uint32_t flags, void *stream, hsla_pattern **out);
void hsla_pattern_destroy(hsla_pattern *p);
/* The rule hsla_pattern_create applies, on host memory and without a
 * device (e.g. to check a pattern before uploading it): row_ptr
 * int32[n+1] and col int32[nnz] are host pointers.  HSLA_OK if canonical;
 * HSLA_ERR_INVALID_CSR with *bad_row (nullable) = the first row that breaks
 * it, or -1 when row_ptr[0] != 0 or row_ptr[n] != nnz (checked first, so
 * every row's range is read only after its bounds are known to lie in
 * [0, nnz]); HSLA_ERR_INVALID_ARG for n < 0, nnz out of [0, 2^31 - 1) or a
 * null pointer. */
hsla_status hsla_csr_check(int32_t n, int64_t nnz, const int32_t *row_ptr, const int32_t *col, int32_t *bad_row);
/* n, nnz, nnz of the lower triangle (incl. diagonal), and 1 if the pattern
 * equals its transpose. */
hsla_status hsla_pattern_info(const hsla_pattern *p, int32_t *n, int64_t *nnz, int64_t *nnz_lower,
                              int32_t *pattern_symmetric);
/* SpMV storage forms.  At creation the library also derives, for A, A^T and
 * the lower/upper triangles, an offset-mask form wherever every entry lies
 * on one of at most 16 fixed diagonals (col - row in a fixed set, as for
 * structured-grid stencils): one 16-bit mask per row replaces the 4-byte
 * column index of every entry, cutting the bytes each SpMV streams.
 *   AUTO (default): hsla_spmv walks row tiles with the masks; the solvers
 *     copy the values once per solve into a diagonal-major layout (entry of
 *     row i on diagonal s at [s][i], zeros where a row has none) and run
 *     every SpMV of the iteration as a row-per-thread stream over it.
 *   CSR: column indices and row tiles everywhere.
 *   DIAGONAL: as AUTO, and hsla_spmv also goes through the diagonal-major
 *     copy (one extra pass over the values per call).
 * Every form adds each row's products in ascending column order, so SpMV
 * results are bitwise identical in all of them (for finite x, up to the sign
 * of a zero sum: the diagonal-major copy's paired layout, hsla_info.spmv_paired,
 * reads no row masks and adds an absent entry's stored 0 times a finite x; a
 * non-finite x there can also reach rows that have no entry at its column);
 * a solve's dot products are reduced in an order that depends on the form's
 * grid, so solves agree to rounding. */
typedef enum hsla_format { HSLA_FORMAT_AUTO = 0, HSLA_FORMAT_CSR = 1, HSLA_FORMAT_DIAGONAL = 2 } hsla_format;
/* Selects the form later calls on `p` use; must not run concurrently with
 * calls that use `p`.  HSLA_ERR_INVALID_ARG for an unknown format. */
hsla_status hsla_pattern_set_format(hsla_pattern *p, int32_t format);
/* stencil_in_use: 1 if A's SpMV currently uses the offset-mask form;
 * num_offsets: number of distinct diagonals of A, 0 if A has no such form. */
hsla_status hsla_pattern_format(const hsla_pattern *p, int32_t *stencil_in_use, int32_t *num_offsets);
/* Autotuner result: the SpMV configuration the solvers use on a pattern. */
typedef struct hsla_tuning {
    int32_t form;          /* 0: per-solve diagonal-major copy, 1: row tiles (CSR or row masks),
                              2: the copy's symmetric half form (used for symmetric values)    */
    int32_t blocks_per_cu; /* grid density of the chosen form's SpMV kernel                   */
    double best_us;        /* mean SpMV time of the choice (B systems)                        */
    double default_us;     /* mean SpMV time of the untuned default configuration             */
} hsla_tuning;
/* Times the solvers' SpMV on this pattern for a batch of B systems, on the
 * device and with synthetic values: the diagonal-major forms (offset-mask
 * patterns, unless the CSR format was selected) at 1, 2, 4, 8, 16 blocks per
 * CU (the symmetric half form also at 3) and the row-tile form at 4, 8, 16,
 * 32 blocks per CU, `effort` launches each
 * (1..100).  Stores the fastest in the pattern (later solves on it use it;
 * results do not depend on the choice beyond rounding of dot products) and
 * reports it in `out` (host, may be NULL).  Uses the handle's workspace;
 * must not run concurrently with other calls that use `p`. */
hsla_status hsla_autotune(hsla_handle *h, hsla_pattern *p, int32_t B, int32_t effort, hsla_tuning *out,
                          void *stream);
/* Device copies of the lower triangle, diagonal included, on which FSAI
 * factors and the network's output live ([B][nnz_lower] value arrays follow
 * its entry order): row_ptr_L int32[n+1], col_L int32[nnz_lower] and
 * pos int32[nnz_lower] with pos[k'] = position in A of the entry stored at
 * k' of the lower triangle.  Any output may be NULL. */
hsla_status hsla_pattern_lower(hsla_handle *h, const hsla_pattern *p, int32_t *d_row_ptr_L, int32_t *d_col_L,
                               int32_t *d_pos, void *stream);
/* A 64-bit signature of the pattern (a hash of n, nnz, row_ptr and col taken
 * at creation): equal patterns have equal signatures in any process. */
hsla_status hsla_pattern_signature(const hsla_pattern *p, uint64_t *signature);
/* The SpMV configuration a pattern holds (its defaults, or the autotuner's
 * choice) as a plain record, so that a tuning can be stored (keyed by the
 * signature, batch size and device) and applied to an equal pattern later,
 * e.g. in another process, without timing again.  hsla_pattern_set_tuning
 * returns HSLA_ERR_INVALID_ARG if the signature differs from the pattern's
 * or a field is out of range; it must not run concurrently with calls that
 * use the pattern. */
typedef struct hsla_tune_state {
    uint64_t signature; /* of the pattern the record was taken from                       */
    int32_t tuned;      /* 1 if set by hsla_autotune (or from such a record)              */
    int32_t dia;        /* 1: the diagonal-major copy, 0: row tiles (offset-mask patterns) */
    int32_t dia_cu;     /* blocks per CU of the diagonal-major SpMV (1..64)               */
    int32_t tile_cu;    /* blocks per CU of the row-tile SpMV (1..64)                     */
    int32_t sym;        /* 1: symmetric half form for symmetric values                    */
    int32_t sym_cu;     /* blocks per CU of the half form's SpMV (1..64)                  */
} hsla_tune_state;
hsla_status hsla_pattern_get_tuning(const hsla_pattern *p, hsla_tune_state *out);
hsla_status hsla_pattern_set_tuning(hsla_pattern *p, const hsla_tune_state *in);
/* A coloring of the pattern's columns in which two columns that share a
 * row get different colors (greedy, columns in ascending order, each taking
 * the smallest color free among the columns it shares a row with), so that
 * a Jacobian with this sparsity pattern is recovered from one Jacobian-vector
 * product per color: the product with the indicator of color c holds
 * J_ij at row i for the one column j of color c in that row (the
 * compression of Curtis, Powell and Reid).  d_color (int32[n], device,
 * nullable) receives the colors, *ncolors (host) their number.  Used by the
 * Newton solves with a general residual (Sec. "Adjoint Differentiation",
 * paragraph "Nonlinear systems"). */
hsla_status hsla_pattern_colors(hsla_handle *h, const hsla_pattern *p, int32_t *d_color, int32_t *ncolors,
                                void *stream);
/* Device copies of the transpose: row_ptr_T int32[n+1], col_T int32[nnz] and
 * src int32[nnz] with src[k'] = position in A of the entry stored at k' of
 * A^T (a bijection).  Host-visible only through the copy. */
hsla_status hsla_pattern_transpose(hsla_handle *h, const hsla_pattern *p, int32_t *d_row_ptr_T,
                                   int32_t *d_col_T, int32_t *d_src, void *stream);

/* ------------------------------------------------------------ operations */
/* y = A x for B systems sharing the pattern: values [B][nnz], x and y
 * [B][n] (Eq. forward_spmv with one process).  Each row sums its products
 * in ascending column order. */
hsla_status hsla_spmv(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                      const double *d_x, double *d_y, void *stream);

/* Solves A x = b (the paper's A.solve(b)).  CG (Hestenes-Stiefel, the
 * recurrence of the paper's Algorithm "Distributed CG" on one device) or
 * right-preconditioned BiCGStab (van der Vorst), with Jacobi, FSAI
 * (M^{-1} = G^T G) or no preconditioner.  All recurrences are FP64; only
 * stored FSAI factors are float32.  `info` (host, may be NULL) receives one
 * record.  Status is the system's status. */
hsla_status hsla_solve(hsla_handle *h, const hsla_pattern *p, const double *d_values,
                       const double *d_b, double *d_x, const hsla_opts *opts, hsla_info *info,
                       void *stream);

/* B independent systems on one pattern (values [B][nnz], b and x [B][n]):
 * the paper's batched solve with a shared sparsity pattern (Sec. "Unified
 * Backend Abstraction", paragraph "Typed sparse-tensor hierarchy", and item
 * 3 of the API listing in Sec. "API Examples"), where the per-pattern data
 * is reused across the batch.  The systems are iterated in lock step with a
 * per-system convergence mask: a system stops
 * when its own test passes, and its result does not depend on the others.
 * `infos` (host, may be NULL) receives B records.  Returns the worst status
 * (an error < 0 if any system errs, else the largest warning). */
hsla_status hsla_solve_batched(hsla_handle *h, const hsla_pattern *p, int32_t B,
                               const double *d_values, const double *d_b, double *d_x,
                               const hsla_opts *opts, hsla_info *infos, void *stream);

/* For callers that cannot allocate device memory during a call (serving
 * loops that must not call hipMalloc, harnesses that forbid it): the same
 * solve as hsla_solve_batched -- same kernels, same results bit for bit as
 * a call of hsla_solve_batched with use_graph = 0 -- with the workspace
 * (state records, partials, work vectors, diagonal-major copies) taken from
 * a 64 MiB array that the library holds on each device it runs on until
 * the process ends, instead of from the handle's workspace.  The call
 * allocates no device memory and instantiates no graph (iterations are
 * launched one by one; opts->use_graph is ignored).  B may be 0..1024.  A
 * solve whose workspace would exceed the array (hsla_workspace_size tells
 * what a solve takes), B beyond 1024, or opts->profile set returns
 * HSLA_ERR_INVALID_ARG with the sizes in hsla_last_error, without writing
 * x.  Every such call on one device shares that device's
 * array, which keeps the last call's contents (nothing in it needs to
 * start at zero): calls that overlap on one device -- from several threads,
 * or on handles whose streams are not ordered -- race and must not be
 * made. */
hsla_status hsla_solve_noalloc(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                               const double *d_b, double *d_x, const hsla_opts *opts, hsla_info *infos,
                               void *stream);

/* Adjoint of the solve (Eq. adjoint_linear): solves A^T lambda = gx with the
 * options' method/preconditioner/tolerance (relative to ||gx||), then
 * gb = lambda (float64[n]) and gA[k] = -lambda[row(k)] * x[col(k)] for every
 * stored entry k, in the pattern's entry order (float64[nnz]).  Either
 * output may be NULL.  x must be the converged forward solution.  AUTO uses
 * CG on A when A is symmetric, otherwise BiCGStab on A^T. */
hsla_status hsla_adjoint(hsla_handle *h, const hsla_pattern *p, const double *d_values,
                         const double *d_x, const double *d_gx, double *d_gA, double *d_gb,
                         const hsla_opts *opts, hsla_info *info, void *stream);

/* Batched adjoint over a shared pattern (Eq. adjoint_linear per system;
 * the paper's batched solves keep gradients flowing through the same
 * adjoint path, Sec. "API Examples"): values [B][nnz], x, gx, gb [B][n],
 * gA [B][nnz].  Each system's adjoint solve stops on its own test. */
hsla_status hsla_adjoint_batched(hsla_handle *h, const hsla_pattern *p, int32_t B,
                                 const double *d_values, const double *d_x, const double *d_gx,
                                 double *d_gA, double *d_gb, const hsla_opts *opts,
                                 hsla_info *infos, void *stream);

/* B systems with distinct patterns and sizes (the paper's matrix list with
 * distinct patterns) solved with CG (Jacobi or no preconditioner, x0 = 0),
 * each to its own stop test.  Batches of at least 2^20 rows with a system
 * above 8192 rows, and every batch when opts->persistent is 0, run
 * segmented: per-iteration kernels stream all systems as one block-diagonal
 * operator in 512-row chunks (a chunk never spans two systems) with each
 * system's sums and scalars kept apart.  Other batches run in one persistent
 * launch: workgroups take systems from a queue, largest first.  A system's
 * result does not depend on the rest of the batch.  System s owns rows
 * [row_off[s], row_off[s+1]) of b and x (float64) and entries
 * [nnz_off[s], nnz_off[s+1]) of col (int32, local column indices) and values
 * (float64); its local row pointer (n_s + 1 int32 entries starting at 0)
 * starts at row_ptr[row_off[s] + s].  Offsets are int64[B+1] device arrays
 * starting at 0.  Every local pattern is validated as canonical CSR
 * (HSLA_ERR_INVALID_CSR names the first bad system).  `infos` (host, may be
 * NULL) receives B records; the return value is the worst status. */
hsla_status hsla_solve_ragged(hsla_handle *h, int32_t B, const int64_t *d_row_off, const int64_t *d_nnz_off,
                              const int32_t *d_row_ptr, const int32_t *d_col, const double *d_values,
                              const double *d_b, double *d_x, const hsla_opts *opts, hsla_info *infos,
                              void *stream);

/* The gradient assembly alone: gA[k] = -lambda[row(k)] * x[col(k)] for B
 * systems ([B][n] inputs, [B][nnz] output). */
hsla_status hsla_outer_on_pattern(hsla_handle *h, const hsla_pattern *p, int32_t B,
                                  const double *d_lambda, const double *d_x, double *d_gA,
                                  void *stream);

/* ||b - A x||_2 and ||b||_2 per system (host outputs, B doubles each). */
hsla_status hsla_residual_norms(hsla_handle *h, const hsla_pattern *p, int32_t B,
                                const double *d_values, const double *d_b, const double *d_x,
                                double *res_norm, double *b_norm, void *stream);

/* ------------------------------------------------------------ learned FSAI */
/* A factorized sparse approximate inverse M^{-1} = G^T G with G lower
 * triangular on A's lower pattern (diagonal included) and a positive
 * diagonal, so preconditioned CG stays valid.  The values come from a small
 * message-passing network over A's graph (this project's design; the paper
 * names learned preconditioners as future work).  The network maps the
 * Jacobi-scaled matrix A^ = D^{-1/2} A D^{-1/2} to G^, and G = G^ D^{-1/2}.
 * Parameters are float32, packed as W0[4][64] b0[64], then per layer l = 1..3
 * C_l[4][64] W_l[128][64] b_l[64], then H1[132][32] c1[32] H2[32] c2. */

/* Number of float32 parameters in the packed layout. */
int32_t hsla_mpnn_num_params(void);

/* G^ (float32 [B][nnz_L], lower entries in the pattern's row order) for B
 * systems sharing pattern p, from their values (float64 [B][nnz]) and the
 * packed parameters (float32, device).  Weights and activations are rounded
 * to bfloat16, products accumulate in float32 on the matrix cores.  With
 * keep != 0 the activations stay in the handle for the next
 * hsla_mpnn_backward (one kept forward per handle).  A missing or
 * non-positive diagonal returns HSLA_ERR_ZERO_DIAGONAL. */
hsla_status hsla_mpnn_forward(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                              const float *d_params, float *d_Ghat, int32_t keep, void *stream);

/* Parameter gradients (float32 [num_params], overwritten) of sum(dGhat * G^)
 * for the most recent kept forward of the same pattern and batch. */
hsla_status hsla_mpnn_backward(hsla_handle *h, const hsla_pattern *p, int32_t B, const float *d_dGhat,
                               float *d_grads, void *stream);

/* Probe loss of the factor: loss[s] = scale * sum_p ||G^ A^ G^^T z_p - z_p||^2
 * for each system s (host output, B doubles) with probes Z (float64
 * [B][P][n], device), FP64 arithmetic on float32 factor values; d_dGhat
 * (float32 [B][nnz_L], nullable) receives the gradient of loss[s] with
 * respect to G^ of system s.  B * P must not exceed 65535. */
hsla_status hsla_probe_loss(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                            const float *d_Ghat, int32_t P, const double *d_Z, double scale, double *loss,
                            float *d_dGhat, void *stream);

/* One Adam step on n float32 parameters (bias-corrected, step >= 1). */
hsla_status hsla_adam_step(hsla_handle *h, int64_t n, float *d_params, const float *d_grads, float *d_m,
                           float *d_v, float lr, float beta1, float beta2, float eps, int64_t step, void *stream);

/* The factors hsla_solve applies with HSLA_PRECOND_FSAI: G = G^ D^{-1/2}
 * (float32 [B][nnz_L]) and the same values in G^T's CSR order (d_GT). */
hsla_status hsla_fsai_factors(hsla_handle *h, const hsla_pattern *p, int32_t B, const double *d_values,
                              const float *d_Ghat, float *d_G, float *d_GT, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HSLA_H */
