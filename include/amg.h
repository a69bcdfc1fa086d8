/*
 * amg.h -- C ABI of libamg.so: unsmoothed-aggregation algebraic multigrid on one
 * AMD MI355X (gfx950), after Brannick, Chen, Hu, Zikatanov, "Parallel Unsmoothed
 * Aggregation Algebraic Multigrid Algorithms on GPUs".
 *
 * Problem (Sec. 2, eq. (2.1)): solve A u = f for a symmetric positive definite
 * weighted graph Laplacian A given in CSR.
 *
 * Conventions for every entry point:
 *   - Pointers to matrices and vectors are DEVICE pointers (for example
 *     torch.Tensor.data_ptr() of a CUDA/HIP tensor) unless the name ends in
 *     _host.  Indices are 0-based int32; values are IEEE binary64.
 *   - Calls are ordered on the stream given in amg_options.stream (NULL: the
 *     library creates its own blocking stream, which is ordered after work on the
 *     legacy default stream).  Calls that return data or status to the host block
 *     until that data is ready.
 *   - No C++ exception crosses this boundary; failures are reported as amg_status.
 *   - A hierarchy must not be used by two host threads at once.
 */
#ifndef UA_AMG_H
#define UA_AMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    AMG_OK = 0,
    AMG_ERR_INVALID_ARGUMENT = 1, /* NULL pointer, bad option, non-finite b          */
    AMG_ERR_INVALID_MATRIX = 2,   /* CSR malformed, diagonal missing or <= 0        */
    AMG_ERR_OUT_OF_MEMORY = 3,    /* device allocation failed or mem_budget exceeded */
    AMG_ERR_DEVICE = 4,           /* a HIP runtime call failed                       */
    AMG_ERR_NOT_CONVERGED = 5,    /* max_iters reached; info holds the last residual */
    AMG_ERR_BREAKDOWN = 6,        /* a Krylov step met p^T A p <= 0: A is not SPD     */
    AMG_ERR_UNSUPPORTED = 7       /* option value outside what is implemented         */
} amg_status;

typedef enum {
    AMG_PREC_FP64 = 0,       /* every level and the K-cycle in binary64                 */
    AMG_PREC_FP32_INNER = 1  /* K-cycle in binary32 inside the binary64 outer iteration */
} amg_precision;

typedef enum {
    AMG_SMOOTHER_L1 = 0,     /* l1-Jacobi, M_ii = a_ii + sum_{j != i} |a_ij| (Sec. 4.1)  */
    AMG_SMOOTHER_JACOBI = 1  /* damped Jacobi, M^-1 = omega D^-1 (Sec. 4.1)            */
} amg_smoother;

/* Opaque hierarchy: owns copies of every level and all its device memory. */
typedef struct amg_hierarchy amg_hierarchy;

/* Square n x n matrix in CSR (device pointers).  Columns strictly ascending in
 * every row, diagonal entry present and > 0 (Sec. 2: positive weights). */
typedef struct {
    int32_t n;
    int32_t nnz;
    const int32_t *row_ptr; /* n + 1 */
    const int32_t *col_idx; /* nnz   */
    const double *values;   /* nnz   */
} amg_csr;

typedef struct {
    int32_t coarsest_size;      /* n_0 of Alg. 1: coarsen while n_l > n_0 (default 64)       */
    int32_t max_levels;         /* L of Alg. 1 (default 40, at most 64)                      */
    double stall_ratio;         /* stop when an aggregation keeps > ratio*n_l (default 0.9)  */
    int32_t max_aggregate;      /* size limit t of Sec. 3.3 / 5.1; 0 = unlimited (default)   */
    uint64_t seed;              /* seed of rand() in eq. (3.2)                               */
    int32_t kcycle_inner;       /* inner flexible-CG steps per coarse visit, 1 or 2 (def. 2) */
    int32_t precision;          /* amg_precision (default AMG_PREC_FP64)                     */
    int32_t max_iters;          /* outer iterations (default 200)                            */
    int32_t max_coarsest;       /* largest coarsest level factored densely (default 4096)   */
    int32_t use_graph;          /* 1: replay the K-cycle as a captured HIP graph (default); */
                                /* 0: launch its kernels one by one (same results)          */
    size_t mem_budget;          /* device bytes the hierarchy may hold; 0 = no limit        */
    void *stream;               /* hipStream_t, or NULL                                      */
    int32_t max_rhs;            /* right-hand sides one amg_solve_batch may take (def. 1);   */
                                /* work vectors are sized n_l * max_rhs on every level       */
    int32_t smoother;           /* amg_smoother of every level (default AMG_SMOOTHER_L1)     */
    double jacobi_weight;       /* omega of AMG_SMOOTHER_JACOBI, finite and > 0 (def. 2/3)  */
    int32_t autotune;           /* 1: at the first solve, time the candidate lanes per row   */
                                /* of levels >= 100k rows and keep the fastest (cached per  */
                                /* level shape and right-hand-side count; default);         */
                                /* 0: lanes from the mean row length                        */
    double kcycle_threshold;    /* theta >= 0 of the K-cycle (Sec. 4.3): the second inner    */
                                /* step of a coarse visit is skipped when the residual after */
                                /* the first is below theta times the restricted residual   */
                                /* (Euclidean norms); 0 = always kcycle_inner steps (def.)  */
    double skip_ratio;          /* level skipping (Sec. 3.3): a level whose aggregation      */
                                /* coarsens by less than this ratio is aggregated twice and */
                                /* the intermediate level dropped; 0 = never (default)      */
    int32_t post_fused;         /* post-smoothing of a level with a sliced copy: 0 = two    */
                                /* launches (the iterate stored), 1 = one sweep forming the */
                                /* iterate per entry, -1 = timed at the first solve with    */
                                /* autotune (default; two launches without).  Same result.  */
    int32_t batch_cols;         /* batched solves on levels >= 100k rows kept in CSR: the    */
                                /* right-hand sides one block serves, each entry loaded     */
                                /* once for all of them (CSR SpMM): 1, 2, 4 or 8; 0 = timed */
                                /* at the first batched solve with autotune, else 4 (def.). */
                                /* Same result for every choice.                            */
} amg_options;

typedef struct {
    int32_t iterations;   /* outer flexible-CG iterations                     */
    double rel_residual;  /* true ||b - A x||_2 / ||b||_2 at return (binary64) */
    double setup_ms;      /* device time of amg_setup for this hierarchy       */
    double solve_ms;      /* device time of this amg_solve                     */
} amg_solve_info;

/* Fills *opt with the defaults listed above. */
void amg_default_options(amg_options *opt);

/* Setup phase of Alg. 1: builds the level hierarchy of A.  Per level: priorities
 * of eq. (3.2), the parallel aggregation of Alg. 2 (Sec. 3.1-3.2), aggregates
 * numbered by increasing coarse-vertex index (Sec. 5.1), the coarse matrix of
 * eq. (2.4) and the l1-Jacobi diagonal (Sec. 4.1); the coarsest level is factored
 * densely.  A is copied: the caller may free its arrays on return.  opt may be
 * NULL (defaults).  On AMG_OK *out receives a hierarchy to release with amg_free;
 * on any error *out is set to NULL and nothing stays allocated. */
amg_status amg_setup(const amg_csr *A, const amg_options *opt, amg_hierarchy **out);

/* Solve phase: outer nonlinear (flexible) preconditioned CG preconditioned by
 * the K-cycle of Sec. 4.3-4.4, stopping when the true relative residual
 * ||b - A x|| / ||b|| <= tol.  b and x are device vectors of length n; x holds the
 * initial guess on entry and the solution on return (written on AMG_OK and
 * AMG_ERR_NOT_CONVERGED).  info (may be NULL) is filled on those two statuses.
 * The K-cycle visits level k nu^k times (nu = kcycle_inner); a hierarchy whose
 * cycle would make more than 65,536 level visits per application (nu = 2 and more
 * than 17 levels) is refused with AMG_ERR_UNSUPPORTED before any launch (raise
 * coarsest_size, lower max_levels or take nu = 1).  The same holds for
 * amg_solve_batch and amg_kcycle. */
amg_status amg_solve(amg_hierarchy *h, const double *b, double *x, double tol, amg_solve_info *info);

/* Solves A X = B for nrhs right-hand sides at once (1 <= nrhs <= opt.max_rhs): every
 * kernel of the K-cycle and of the outer iteration serves all columns in one
 * launch (grid dimension y = column).  B and X are column-major device arrays, column
 * c at B + c * ldb and X + c * ldx (ldb, ldx >= n); X holds the initial guesses on
 * entry.  Each column is iterated until its own recursive and true relative
 * residuals are <= tol (columns that converge early keep iterating with the others;
 * a zero right-hand side gives X = 0).  info (may be NULL) receives nrhs records,
 * written on AMG_OK and AMG_ERR_NOT_CONVERGED; iterations is the iteration at which
 * each column was confirmed.  One column gives the same result as amg_solve. */
amg_status amg_solve_batch(amg_hierarchy *h, int32_t nrhs, const double *B, int32_t ldb, double *X, int32_t ldx,
                           double tol, amg_solve_info *info);

/* ---- Grouped solves of small problems (one launch for many requests) ----
 * One right-hand side of one hierarchy: solve A x = b of h.  column (0 <= column <
 * h's max_rhs) names the set of h's work vectors the job uses; two jobs of one call
 * on the same hierarchy must name different columns.  b and x are device vectors of
 * h's n unknowns in the caller's numbering; x holds the initial guess on entry.
 * b and x must not overlap. */
typedef struct {
    amg_hierarchy *h;
    int32_t column;
    const double *b;
    double *x;
} amg_group_job;

/* Solves `count` jobs -- on different hierarchies, of different sizes and depths, or
 * several right-hand sides of one -- in ONE kernel launch: one workgroup runs the
 * whole outer flexible CG (Sec. 4.4) with its K-cycle preconditioner (Sec. 4.3, the
 * hierarchy's kcycle_inner, kcycle_threshold and smoother) for one job, so the
 * latency-bound small levels of concurrent requests share a dispatch instead of
 * taking thousands each.  Meant for small problems (a workgroup sweeps a level at
 * the bandwidth of one compute unit); the method and stopping rule are those of
 * amg_solve (recursive relative residual <= tol, confirmed by the true residual,
 * the iteration continuing from the true residual when it disagrees), with
 * h's max_iters.  Each job's sums run in a fixed order that does not depend on the
 * other jobs: a job gives the same bits alone and in any group.  The result is
 * not bit-identical to amg_solve's (other summation orders), and agrees with it to
 * the tolerance.
 *   Requirements (else AMG_ERR_UNSUPPORTED before any launch): every hierarchy in
 * AMG_PREC_FP64, with 2 to 16 levels and within the visit budget of amg_solve.
 * Argument errors (NULL job arrays, b or x not device memory, a column out of
 * range or repeated on one hierarchy, tol not finite and > 0): AMG_ERR_INVALID_ARGUMENT.
 * The call waits for each hierarchy's own stream, launches on `stream` (hipStream_t;
 * NULL: the stream of jobs[0].h), and returns when every job is done.  status[k]
 * receives job k's status (AMG_OK, AMG_ERR_NOT_CONVERGED, AMG_ERR_BREAKDOWN, or
 * AMG_ERR_INVALID_ARGUMENT for a non-finite b or x); info (may be NULL) receives
 * count records (solve_ms: device time of the whole launch).  Returns AMG_OK when
 * every job converged, else the first failing job's status.  The hierarchies must
 * not be in use by other calls meanwhile. */
amg_status amg_solve_group(int32_t count, const amg_group_job *jobs, double tol, void *stream, int32_t *status,
                           amg_solve_info *info);

/* x = B b for every job: one application of the K-cycle preconditioner of the
 * job's hierarchy (Sec. 4.3) per job, run as in amg_solve_group (one workgroup per
 * job, one launch).  Same requirements and argument rules; status[k] is AMG_OK or
 * AMG_ERR_BREAKDOWN. */
amg_status amg_kcycle_group(int32_t count, const amg_group_job *jobs, void *stream, int32_t *status);

/* ---- Synthetic workload (the benchmarks' inputs, built in device memory) ----
 * The (2d+1)-point finite-difference Laplacian on the interior of a d-dimensional
 * grid (d = 1, 2, 3; dims[a] >= 1 interior nodes along axis a; unknowns numbered x
 * fastest), Dirichlet boundary, edge weights 1 + jitter (2u - 1) with u drawn by
 * SplitMix64 from `seed` (the model problem of Sec. 2).  Bit-identical to the host
 * generator of the Python package.  row_ptr (n + 1), col_idx and values
 * (amg_grid_laplacian_nnz entries) are device arrays owned by the caller; the call
 * is ordered on `stream` (hipStream_t or NULL) and returns when the arrays are
 * written.  amg_grid_laplacian_nnz returns -1 for invalid dimensions. */
int64_t amg_grid_laplacian_nnz(int32_t dim, const int32_t *dims);
amg_status amg_grid_laplacian(int32_t dim, const int32_t *dims, double jitter, uint64_t seed, int32_t *row_ptr,
                              int32_t *col_idx, double *values, void *stream);
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops that forbid hipMalloc): the same grid Laplacian as
 * amg_grid_laplacian, bit for bit, with no allocation of any kind.  The scan of the
 * row pointers uses a scratch array that the library holds in static device memory
 * (256 KiB per GPU, kept until the process ends), so grids are limited to
 * 134,217,728 (2^27) unknowns; larger valid grids return AMG_ERR_UNSUPPORTED before
 * any device work.  Asynchronous: the arrays are written in order on `stream`, which
 * must belong to the current device; the call does not wait.  Every call on one GPU
 * shares that GPU's scratch, so calls whose work overlaps on the device (different
 * streams without ordering between them) race and must not be made; calls ordered
 * on one stream are safe.  Argument errors as amg_grid_laplacian. */
amg_status amg_grid_laplacian_noalloc(int32_t dim, const int32_t *dims, double jitter, uint64_t seed,
                                      int32_t *row_ptr, int32_t *col_idx, double *values, void *stream);
/* out[i] = 2 u_i - 1 with u_i the i-th SplitMix64 uniform of `seed` (device array of n,
 * ordered on `stream`, asynchronous). */
amg_status amg_uniform_rhs(int64_t n, uint64_t seed, double *out, void *stream);

/* Releases every resource of h.  NULL is accepted.  Device blocks are kept in a
 * process-wide cache (per device and size class) for later hierarchies, because
 * returning memory to the driver synchronises the device; see
 * amg_release_cached_memory. */
void amg_free(amg_hierarchy *h);

/* Returns every cached device block to the driver.  Blocks in use by live
 * hierarchies are not affected.  An allocation that the driver refuses does this
 * by itself before it fails.  Call it with no solve in flight on any stream. */
void amg_release_cached_memory(void);

/* Device bytes the hierarchy holds (matrices, layouts, work vectors, inner-product
 * sites) -- the figure a caller admitting work by memory footprint accounts. */
amg_status amg_memory_bytes(const amg_hierarchy *h, size_t *bytes);

/* Number of levels (finest = 0, coarsest = levels - 1). */
amg_status amg_num_levels(const amg_hierarchy *h, int32_t *levels);

/* Size of level `level`: unknowns, stored entries, and the number of passes of
 * Alg. 2 that aggregated it (0 on the coarsest level).  NULL outputs are skipped. */
amg_status amg_level_sizes(const amg_hierarchy *h, int32_t level, int32_t *n, int32_t *nnz, int32_t *passes);

/* Slots (stored entries, padding included) of the sliced ELLPACK copy that the
 * solve sweeps of level `level` read (slices of 64 rows stored column-major;
 * kept on levels of at least 100k rows whose row lengths vary little), or 0 when
 * the level is swept in CSR only. */
amg_status amg_level_slots(const amg_hierarchy *h, int32_t level, int64_t *slots);

/* Copies level `level` to host arrays in the natural (aggregation) numbering:
 * agg_host[n] = coarse index of each unknown (column of P, eq. (2.2); -1 on the
 * coarsest level), row_ptr_host[n+1], col_host[nnz], val_host[nnz].  Any output
 * may be NULL. */
amg_status amg_export_level(const amg_hierarchy *h, int32_t level, int32_t *agg_host, int32_t *row_ptr_host,
                            int32_t *col_host, double *val_host);

/* y = A_level x for device vectors in the natural numbering of that level (the
 * sparse product of Sec. 4.4). */
amg_status amg_spmv(amg_hierarchy *h, int32_t level, const double *x, double *y);

/* z = B r: one application of the K-cycle preconditioner on the finest level
 * (Sec. 4.3), device vectors of length n in the natural numbering. */
amg_status amg_kcycle(amg_hierarchy *h, const double *r, double *z);

/* Z = B R for nrhs columns at once (1 <= nrhs <= opt.max_rhs), every kernel serving
 * all columns in one launch as in amg_solve_batch: column c of R at R + c * ldr and
 * of Z at Z + c * ldz (ldr, ldz >= n), device memory, natural numbering.  Each column
 * takes its own decisions (the K-cycle threshold), so column c equals amg_kcycle on
 * it alone. */
amg_status amg_kcycle_batch(amg_hierarchy *h, int32_t nrhs, const double *R, int32_t ldr, double *Z, int32_t ldz);

/* Average device time in microseconds of the finest level's post-smoothing step
 * as the solve runs it (prolongation of the coarse correction + one smoothing
 * sweep, Sec. 4.2-4.3, with the inner product (z, A p) of the outer flexible CG
 * in the FP64 mode; two launches on levels of at least 100k rows, one fused
 * launch below), measured with events over `reps` back-to-back steps on the
 * hierarchy's stream; *bytes receives the step's algorithmic DRAM traffic.
 * AMG_ERR_UNSUPPORTED below 3 levels or before the first solve or K-cycle
 * application (the step reads that K-cycle's inner products). */
amg_status amg_time_smoother(amg_hierarchy *h, int32_t reps, double *avg_us, double *bytes);

/* Human-readable name of a status code (static storage). */
const char *amg_status_string(amg_status s);

#ifdef __cplusplus
}
#endif

#endif /* UA_AMG_H */
