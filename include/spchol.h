/*
 * spchol.h -- C ABI of the MI355X supernodal sparse Cholesky library.
 *
 * The library follows the three phases of a direct solver (paper Sec. 1 and
 * Sec. 2, "Background on CHOLMOD"): analyze the pattern of an SPD matrix,
 * factorize A = L L^T numerically, solve L y = b and L^T x = y.  The numeric
 * phases run in hand-written HIP kernels for gfx950; analyze runs on the host.
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int status (enum spc_status); no exception or
 *     C++ type crosses this boundary.
 *   - Indices are 0-based.  A matrix is given as its lower triangle,
 *     diagonal included, in compressed-column form: colptr int64[n+1],
 *     rowidx int32[nnz] (rows strictly increasing inside a column, first row
 *     of column j equal to j), values double[nnz] in the same order.
 *   - Pointers named h_* are host memory, d_* are device memory on the
 *     current HIP device.  The library never frees caller memory.  Handles
 *     are created by the library and released by the caller with the
 *     matching spc_free_* function; freeing NULL is a no-op.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Numeric calls are asynchronous on it; numeric failure (a non-positive
 *     pivot) is reported by spc_sync.
 *   - One handle must not be used from two host threads at once, and the
 *     work of two calls on one factor must not overlap on the device (a
 *     factor owns one solve workspace): queue them on one stream, or wait
 *     for one before issuing the other on another stream.  Distinct handles
 *     may be used concurrently on distinct streams.
 */
#ifndef SPCHOL_H
#define SPCHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum spc_status {
    SPC_OK = 0,
    SPC_INVALID_INPUT = -1,   /* malformed CSC / permutation / argument */
    SPC_NOT_SPD = -2,         /* a pivot was not positive and finite */
    SPC_OUT_OF_MEMORY = -3,   /* device or host allocation failed */
    SPC_NO_CONVERGENCE = -4,  /* refinement did not reach the tolerance */
    SPC_DEVICE_ERROR = -5,    /* a HIP call failed, or a device-side wait gave up */
    SPC_BAD_HANDLE = -6,      /* NULL or already released handle */
    SPC_NO_DEVICE = -7        /* no usable gfx950 device */
};

enum spc_precision {
    SPC_FP64 = 0,             /* panels, updates and solves in double */
    SPC_FP32 = 1,             /* panels, updates and solves in float, float accumulation */
    SPC_FP32_BF16UPD = 2      /* as SPC_FP32, but the SYRK/GEMM Schur-complement updates of the
                               * tiled paths (the trailing update inside a wide supernode, except
                               * the diagonal tile of the block factored next, and the scatter
                               * updates into ancestors) multiply operands rounded to BF16 on
                               * BF16 MFMA with FP32 accumulation; POTRF, TRSM, the block
                               * inverses, the small-supernode paths and the solves stay FP32.
                               * Not in the paper: an experiment in how little precision the
                               * updates need when FP64 refinement (spc_solve_refined) follows. */
};

typedef struct spc_symbolic_s *spc_symbolic;
typedef struct spc_factor_s *spc_factor;
typedef struct spc_batch_s *spc_batch;

/* Analysis options.  Pass NULL for the defaults. */
typedef struct spc_options {
    /* Chain amalgamation tolerance z: a supernode absorbs its only
     * predecessor chain while the explicit zeros stay within z of the stored
     * entries (paper Sec. 2 describes node amalgamation; the exact rule is
     * this library's).  z < 0 keeps the fundamental supernodes; NaN gives
     * SPC_INVALID_INPUT.  Default 0.05. */
    double amalg_z;
    /* Schedule cut-offs (the choice between batching small supernodes of a
     * level into one launch and giving a large one the whole device).
     * 0 keeps the library default, a negative value turns the path off.
     *   tiny_w, tiny_m    supernodes with w <= tiny_w and m <= tiny_m are
     *                     factored (and solved in the wide levels) one wave
     *                     each; at most 8 and 64 (default 8, 64)
     *   small_w, small_m  the same limits for one workgroup each; at most 32
     *                     and 128 (default 32, 128)
     *   big_min, big_min_k  scatter updates with m - w >= big_min and
     *                     w >= big_min_k use 128x128 tiles (default 256, 128)
     *   solve_persist_max  solve levels from the top with fewer tasks than
     *                     this run as one persistent launch per sweep
     *                     (default 1024)
     *   handover          1: inside a wide supernode, the tiles below a
     *                     64-column block that its trailing launch factors
     *                     take the block's TRSM in the same launch, waiting
     *                     on device flags for its panels; a negative value
     *                     gives every block a TRSM launch of its own (no
     *                     waits inside a launch: for many factorizations
     *                     sharing the device on several streams); 2 keeps
     *                     the hand-over only in steps where few tiles wait
     *                     (eight or more supernodes, or the waiting tiles at
     *                     most 1.5 of a launch's mean share per XCD beside
     *                     the step's other tiles), the others get a TRSM
     *                     launch.  Default 1.
     *   delay             column blocks per bulk trailing update inside a wide
     *                     supernode: the columns beyond a group of `delay`
     *                     64-column blocks receive the group's update once,
     *                     with K = 64 * delay, while each next block inside
     *                     the group is brought up to date on its own; at most
     *                     8 (default 1; a negative value keeps 1)
     *   persist           1: every small subtree (a supernode whose whole
     *                     subtree is within the one-wave or one-workgroup
     *                     limits), of every system of a batch, is factored by
     *                     one persistent launch across all its levels, with
     *                     device-side dependency counters; a negative value
     *                     (the default, 0) launches those supernodes level by
     *                     level, which measured faster on the workloads here.
     *   ordering          when spc_analyze gets no order (h_perm NULL): 0
     *                     the identity (default), 1 graph nested dissection,
     *                     2 minimum degree (see spc_order)
     *   group             1 (default): tiny supernodes with w <= 4 and
     *                     m <= 16 (m <= 32) share a wave, 16 (32) lanes
     *                     each; a negative value gives each its own wave
     *   bulk128           1: the bulk trailing updates inside a wide
     *                     supernode (K = 64 * delay >= 128) run on 128x128
     *                     tiles in a launch of their own; a negative value
     *                     (the default, 0) keeps them on 64x64 tiles in the
     *                     step's trailing launch
     *   lookahead         1 (with delay >= 2): a group's bulk update reaches
     *                     only the next group's columns at once; the columns
     *                     beyond get it in the next group's other steps,
     *                     beside their column updates and factorizations; a
     *                     negative value (the default, 0) updates them all
     *                     at the end of the group
     * Values beyond a kernel's limit give SPC_INVALID_INPUT. */
    int32_t tiny_w, tiny_m, small_w, small_m;
    int32_t big_min, big_min_k, solve_persist_max;
    int32_t handover;
    int32_t delay;
    int32_t persist;
    int32_t ordering;
    int32_t group;
    int32_t bulk128;
    int32_t lookahead;
    /* Device-memory budget in bytes for each factorization of this analysis
     * (the footprint spc_symbolic_info reports as factor_bytes_fp64 or
     * factor_bytes_fp32, by precision; a batch is held to the smallest
     * positive budget among its members, over the merged footprint).  A
     * factorization or batch that would exceed it is refused with
     * SPC_OUT_OF_MEMORY before anything is allocated, and
     * spc_last_error_message names both sizes.  0 or negative: no budget
     * (default).  Admission by footprint is the memory side of the paper's
     * per-phase analysis (Sec. 2: the symbolic phase fixes the storage of
     * L before any numeric work). */
    int64_t hbm_budget;
} spc_options;

/* Summary numbers of an analysis. */
typedef struct spc_info {
    int64_t n;
    int64_t nnz_a;            /* entries of the lower triangle given */
    int64_t nsuper;           /* supernodes after amalgamation */
    int64_t nnz_l;            /* sum of column counts (exact pattern of L) */
    int64_t panel_entries;    /* stored panel entries, sum of m_s * w_s */
    int64_t flops;            /* sum of squared column counts */
    int64_t levels;           /* height of the supernodal elimination tree */
    int64_t rows_total;       /* sum of |R_s| */
    int64_t max_width;        /* widest supernode */
    int64_t max_rows;         /* longest row list */
    int64_t factor_bytes_fp64;/* device bytes of an FP64 factor + plan */
    int64_t factor_bytes_fp32;/* device bytes of an FP32 factor + plan */
    int64_t solve_levels;     /* levels of the column-block tree the solves sweep */
    int64_t solve_persistent_levels; /* top levels run as one persistent launch per sweep */
    int64_t solve_block_tasks;/* row tasks of the block solve kernels */
    int64_t solve_tiny_tasks; /* tiny supernodes solved one wave each */
    int64_t updates_total;    /* sum of |U_s|: (source, ancestor) update pairs */
    int64_t solve_handovers;  /* pairs of consecutive blocks of a supernode that the
                                 persistent solve sweeps hand over directly */
} spc_info;

/*
 * spc_analyze -- symbolic phase (paper Sec. 2: reordering, elimination tree,
 * node amalgamation into supernodes).  Host only; touches no device.
 *   n        matrix order (>= 0)
 *   h_colptr, h_rowidx   lower CSC pattern as described above
 *   h_perm   fill-reducing order, perm[k] = original index of pivot k, or
 *            NULL for the identity.  The library composes it with a
 *            postorder of the elimination tree.
 *   opts     NULL or options
 *   out      receives the handle
 * Errors: SPC_INVALID_INPUT for any malformed input (unsorted or duplicate
 * rows, entries above the diagonal, a missing diagonal, out-of-range
 * indices, perm not a permutation), SPC_OUT_OF_MEMORY.
 */
int spc_analyze(int64_t n, const int64_t *h_colptr, const int32_t *h_rowidx,
                const int32_t *h_perm, const spc_options *opts, spc_symbolic *out);

int spc_symbolic_info(spc_symbolic sym, spc_info *out);

/*
 * spc_order -- a fill-reducing order of a pattern without coordinates (paper
 * Sec. 2: the analysis reorders the matrix to reduce fill, with METIS or
 * AMD; these are this library's own methods).  Host only.
 *   n, h_colptr, h_rowidx   lower CSC pattern (as for spc_analyze)
 *   method   0 identity; 1 graph nested dissection: in each connected part a
 *            breadth-first level structure from a pseudo-peripheral vertex,
 *            the separator a level with the fewest vertices that leaves at
 *            least a third of the part on each side (thinned to the vertices
 *            touching the next level), both sides recursively, then the
 *            separator; parts of at most 64 vertices by minimum degree;
 *            2 minimum degree on the elimination graph (exact degrees, ties
 *            to the lowest index; n <= 10,000)
 *   h_perm   receives perm[k] = the original index of the k-th pivot, the
 *            form spc_analyze takes
 * Errors: SPC_INVALID_INPUT (malformed pattern, unknown method, minimum
 * degree above its size limit), SPC_OUT_OF_MEMORY.
 */
int spc_order(int64_t n, const int64_t *h_colptr, const int32_t *h_rowidx, int method, int32_t *h_perm);

/* Check the device schedule of an analysis on the host (no device needed),
 * for tests and diagnostics: every 64-column block of the blocked path has
 * the rows below its diagonal solved exactly once (by a TRSM launch, or by
 * the hand-over tiles of the step before, spc_options.handover), and every
 * tile that waits inside a trailing launch comes after the diagonal tile of
 * its block and carries the task that tile runs: the block's factorization
 * is claimed by the first of those workgroups to start, so a wait is only
 * ever on a running workgroup.  Returns SPC_OK, or SPC_INVALID_INPUT with the
 * first violation in spc_last_error_message(); SPC_BAD_HANDLE for a bad
 * handle. */
int spc_symbolic_verify(spc_symbolic sym);

/* Export one symbolic array to host memory for inspection.
 *   0 perm int32[n]        final order (given order composed with postorder)
 *   1 parent int32[n]      elimination tree of the permuted matrix, -1 root
 *   2 colcount int32[n]    column counts of L, diagonal included
 *   3 super_ptr int32[nsuper+1]  first column of each supernode
 *   4 sparent int32[nsuper]      supernodal parent, -1 root
 *   5 rptr int64[nsuper+1]       row-list offsets
 *   6 rows int32[rows_total]     row lists R_s (sorted; first w_s are cols(s))
 *   7 lptr int64[nsuper+1]       panel offsets (m_s*w_s entries each)
 *   8 level int32[nsuper]        0 for leaves, else 1 + max over children
 *   9 uptr int64[nsuper+1]       offsets of the update lists U_s
 *  10 ulist int32[updates_total] U_s: every supernode d < s with a row of R_d
 *                                among cols(s), ascending (Sec. 3, Listing 1)
 * Returns SPC_INVALID_INPUT for an unknown `which`. */
int spc_symbolic_export(spc_symbolic sym, int which, void *h_dst);

/*
 * spc_factorize -- numeric phase (paper Sec. 3, Listing 1: per supernode the
 * SYRK/GEMM updates from earlier supernodes, then POTRF and TRSM).  The
 * device schedule is right-looking by elimination-tree level: every
 * supernode of one level is factored in batched launches, then its
 * Schur-complement update is scatter-added into its ancestors through
 * relative indices.
 *   d_values  device double[nnz] in the CSC order given to spc_analyze
 *   precision enum spc_precision
 *   stream    hipStream_t or NULL
 *   out       receives a factor handle that owns its device storage
 * Asynchronous; call spc_sync to learn whether the matrix was SPD.
 */
int spc_factorize(spc_symbolic sym, const double *d_values, int precision, void *stream,
                  spc_factor *out);

/* Re-run the numeric phase into an existing factor (same pattern, new
 * values); allocates nothing once the factor exists. */
int spc_refactorize(spc_factor f, const double *d_values, void *stream);

/*
 * spc_factorize_batch -- factor `count` independent systems in one
 * level-scheduled pass: the launches of level l carry the supernodes of
 * level l of every system (the systems form one elimination forest; paper
 * Sec. 3 schedules independent supernodes of the tree together).
 * Arguments as for spc_factorize, one per system; all systems use
 * `precision` and `stream`.  outs[i] receives a view of system i's factor
 * (usable with spc_solve, spc_solve_refined, spc_sync, spc_factor_export;
 * not with spc_refactorize); the views share one allocation, released when
 * the last view is freed.  Equivalent to spc_batch_create +
 * spc_batch_factorize + spc_batch_factor for every system.
 */
int spc_factorize_batch(int count, const spc_symbolic *syms, const double *const *d_values,
                        int precision, void *stream, spc_factor *outs);

/*
 * Batch handle: the disjoint union of `count` analyses with one device
 * schedule, created once and factored / solved repeatedly.
 *   spc_batch_create     merge the analyses (host) and allocate the merged
 *                        factor on the device; the batch keeps references to
 *                        the symbolic handles
 *   spc_batch_factorize  d_values[i]: system i's values (device, caller CSC
 *                        order); one level-scheduled pass over all systems
 *   spc_batch_factor     a view of system i's factor (free with
 *                        spc_free_factor)
 *   spc_batch_solve      d_B[i]: system i's right-hand sides (device, n_i x
 *                        nrhs column-major, leading dimension ldb[i] >= n_i,
 *                        host arrays d_B and ldb), solved in place by one
 *                        level-scheduled pass; returns after the stream has
 *                        drained
 *   spc_batch_sync       SPC_NOT_SPD with the first failing system and its
 *                        permuted pivot column, else SPC_OK
 */
int spc_batch_create(int count, const spc_symbolic *syms, int precision, spc_batch *out);
int spc_batch_factorize(spc_batch b, const double *const *d_values, void *stream);
int spc_batch_factor(spc_batch b, int i, spc_factor *out);
int spc_batch_solve(spc_batch b, double *const *d_B, int nrhs, const int64_t *ldb, void *stream);
int spc_batch_sync(spc_batch b, int64_t *bad_system, int64_t *bad_pivot);
int spc_batch_last_ms(spc_batch b, float *ms);
int spc_batch_info(spc_batch b, spc_info *out);
void spc_free_batch(spc_batch b);

/*
 * spc_solve -- X := A^{-1} B in place (paper Sec. 2: the two triangular
 * systems L y = b and L^T x = y).
 *   d_B   device double, n x nrhs column-major with leading dimension ldb,
 *         original (unpermuted) ordering; overwritten with the solution
 * The arithmetic runs in the factor's precision.  Asynchronous.
 */
int spc_solve(spc_factor f, double *d_B, int nrhs, int64_t ldb, void *stream);

/*
 * spc_solve_noalloc -- spc_solve for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same kernels and the same result, but the work
 * vectors live in a fixed scratch array inside the library (64 MiB of device
 * memory per device the library runs on, held until the process ends)
 * instead of the factor's own work area, so the call allocates nothing.
 * The right-hand sides are solved in chunks of as many columns as fit the
 * array (at most 16; 3 * n * 8 bytes per column in FP64, 3 * n * 4 in FP32).
 *   arguments as for spc_solve
 * Every call on one device shares that device's array: calls that overlap on
 * the device race (queue them on one stream).  The array keeps the last
 * call's contents; each call clears what it needs.
 * Errors: as spc_solve; SPC_INVALID_INPUT (with spc_last_error_message) when
 * even one right-hand side does not fit the array.
 */
int spc_solve_noalloc(spc_factor f, double *d_B, int nrhs, int64_t ldb, void *stream);

/* Result of iterative refinement. */
typedef struct spc_refine_info {
    int32_t iterations;       /* refinement steps taken */
    int32_t converged;        /* 1 if berr <= tol */
    double berr;              /* final max-over-RHS normwise backward error */
} spc_refine_info;

/*
 * spc_solve_refined -- solve with the factor, then refine in FP64 on the
 * device: r = b - A x (FP64 sparse product with the original A), d = solve(r)
 * in the factor's precision, x += d (FP64), until the backward error
 *   max_k ||b_k - A x_k||_inf / (||A||_inf ||x_k||_inf + ||b_k||_inf) <= tol
 * or maxit steps.  Once a step cuts that error less than tenfold, conjugate
 * gradients preconditioned by the factor's solve continue from x; after a
 * refined solve that switched, the next ones with the same factorization
 * start with them (a new factorization starts over with the classical
 * steps).  d_values must be the values the factor was built from.
 *   d_B  device double n x nrhs (ld), not modified
 *   d_X  device double n x nrhs (ld), receives the solution
 * Returns SPC_NO_CONVERGENCE (with info filled) when tol is not reached.
 * Synchronizes `stream` once per step to read the error.
 */
int spc_solve_refined(spc_factor f, const double *d_values, const double *d_B, double *d_X,
                      int nrhs, int64_t ld, double tol, int maxit, void *stream,
                      spc_refine_info *info);

/*
 * spc_batch_solve_refined -- spc_solve_refined for every system of a batch
 * at once: one merged solve per step serves all systems, while the norms,
 * the backward error and the conjugate-gradient coefficients are kept per
 * system and right-hand side, so each system converges (and is checked)
 * on its own.  A is the matrix of the last spc_batch_factorize.
 *   d_B[i]  system i's right-hand sides (device, n_i x nrhs column-major,
 *           leading dimension ld[i] >= n_i), not modified
 *   d_X[i]  receives system i's solution (same layout)
 *   infos   nullable host array [count]: per-system result
 * d_B, d_X and ld are host arrays.  Returns SPC_NO_CONVERGENCE if any
 * system missed tol; returns after the stream has drained.
 */
int spc_batch_solve_refined(spc_batch b, const double *const *d_B, double *const *d_X, int nrhs,
                            const int64_t *ld, double tol, int maxit, void *stream,
                            spc_refine_info *infos);

/* Wait for the factor's work on its stream; SPC_NOT_SPD if a pivot failed,
 * with *bad_pivot (nullable) set to the permuted column of the first
 * failing pivot found, else -1.  SPC_DEVICE_ERROR (checked first) if a
 * bounded wait of one workgroup on another gave up during the last
 * factorization or any solve since (see spc_factor_set_wait_limit): the
 * factor and those solutions are then unreliable; the condition stays until
 * the factor is factored again.  spc_solve_refined, spc_batch_solve,
 * spc_batch_solve_refined and spc_batch_sync report it the same way. */
int spc_sync(spc_factor f, int64_t *bad_pivot);

/* SPC_FP32_BF16UPD: the number of pivots of the last factorization (of the
 * whole batch, for a batch view) that were raised to their floor, else 0.
 * With BF16-rounded Schur updates the computed Schur complement of an
 * ill-conditioned matrix can lose definiteness (the rounding perturbs it by
 * about 2^-8 of |L||L^T|); a pivot d_j below theta * a_jj, with theta = 2^-8
 * (BF16's unit roundoff) and a_jj the column's diagonal entry in A, is then
 * replaced by theta * a_jj (static pivot perturbation: the factor is that of
 * A plus a non-negative diagonal), so the factorization completes and the
 * FP64 refinement (whose residual uses A itself) corrects for it.  NaN or
 * Inf pivots still give SPC_NOT_SPD.  Synchronizes. */
int spc_factor_pivot_floors(spc_factor f, int64_t *raised);

/* Polls before a bounded wait of one workgroup on another gives up (the
 * hand-over inside a trailing launch, the persistent solve sweeps).  Every
 * such wait is bounded so that every wave exits whatever happens; one that
 * gives up sets the factor's device-error word, which spc_sync reports as
 * SPC_DEVICE_ERROR.  Default about a second of polls (2^20).  0 makes every
 * wait give up at once: the kernels still run to their end and the results
 * are garbage, which lets a test drive the error path from the host.
 * SPC_INVALID_INPUT for polls < 0 or a batch view. */
int spc_factor_set_wait_limit(spc_factor f, int32_t polls);

/* Copy the panels to host as double (lptr layout of spc_symbolic_export;
 * strict upper triangles of the diagonal blocks are zeroed). Synchronous. */
int spc_factor_export(spc_factor f, double *h_dst);

/* Device time in milliseconds of the last numeric factorization of f,
 * measured with events around its launches on its stream. */
int spc_factor_last_ms(spc_factor f, float *ms);

/* Kernel classes of the numeric phase, for spc_factor_kernel_stats; each
 * class is one kernel (the assemble class: the zero fill and the scatter
 * of A), so per-launch figures of a class are those of its kernel. */
enum spc_kernel_class {
    SPC_K_ASSEMBLE = 0,       /* zero the panels, scatter A into them */
    SPC_K_POTRF = 1,          /* POTRF of 64-column diagonal blocks, with their inverses */
    SPC_K_TRSM = 2,           /* rows below a block times its transposed inverse */
    SPC_K_TRAILING = 3,       /* SYRK/GEMM update inside a wide supernode (64x64 tiles) */
    SPC_K_SCATTER = 4,        /* SYRK/GEMM update scatter-added into ancestors, 64x64 tiles */
    SPC_K_SCATTER_BIG = 5,    /* the same on 128x128 tiles (large supernodes) */
    SPC_K_SMALL = 6,          /* whole small supernodes: POTRF, TRSM, inverse, scatter */
    SPC_K_TINY = 7,           /* the same for tiny supernodes, one wave each */
    SPC_K_SMALL_TREES = 8,    /* the persistent launch over the small subtrees (all their levels) */
    SPC_K_COUNT = 9
};

typedef struct spc_kernel_stats {
    int64_t launches;         /* launches of the class in the last factorization */
    double total_ms;          /* sum of their device durations (events on the stream) */
    double flops;             /* sum of their algorithmic flops (LAPACK counts) */
} spc_kernel_stats;

/* Turn per-launch event timing of f's factorizations on (1) or off (0).
 * While on, every numeric launch is bracketed by two events on the stream. */
int spc_factor_set_profiling(spc_factor f, int on);

/* Graph replay (for callers that refactor the same pattern again and
 * again, e.g. under a launch-bound schedule): on (1), the next factorization
 * of f captures its whole launch sequence into a HIP graph, and later ones
 * replay it with one launch on the given stream; the graph is captured
 * again when the values pointer changes.  Results are those of the eager
 * path.  Profiling (spc_factor_set_profiling) takes the eager path.  Off
 * (0) frees the graph.  A batch view refuses it (SPC_INVALID_INPUT); use
 * spc_batch_set_graph, which covers spc_batch_factorize (the per-system
 * value copies stay outside the graph). */
int spc_factor_set_graph(spc_factor f, int on);
int spc_batch_set_graph(spc_batch b, int on);

/* Per-class totals of the last profiled factorization of f (synchronizes). */
int spc_factor_kernel_stats(spc_factor f, int kernel_class, spc_kernel_stats *out);
int spc_batch_set_profiling(spc_batch b, int on);
int spc_batch_kernel_stats(spc_batch b, int kernel_class, spc_kernel_stats *out);

/* The same totals per elimination-tree level of the schedule (0 = leaves,
 * up to spc_info.levels - 1; -1 = the assembly of A; -2 = the persistent
 * launch over the small subtrees, which spans levels), over all classes. */
int spc_factor_level_stats(spc_factor f, int level, spc_kernel_stats *out);
int spc_batch_level_stats(spc_batch b, int level, spc_kernel_stats *out);

void spc_free_symbolic(spc_symbolic sym);
void spc_free_factor(spc_factor f);
const char *spc_status_string(int status);

/* Text of the last HIP failure seen by this host thread (error string, the
 * failing call and its place), or "" if none.  Owned by the library. */
const char *spc_last_error_message(void);

#ifdef __cplusplus
}
#endif
#endif /* SPCHOL_H */
