/*
 * taskchol.h -- C ABI of the host task-parallel supernodal Cholesky (the
 * paper's own method, used as the strong multicore CPU baseline beside the
 * GPU library; it never runs on the GPU path).
 *
 * The paper (Sec. 3, Listing 1) factors supernodes left-looking: each
 * supernode is an outer task that gathers the SYRK/GEMM updates of the
 * earlier supernodes touching its columns, then runs POTRF and TRSM; outer
 * tasks are ordered by the elimination tree.  Selective nesting (Sec. 4)
 * splits an outer task into one inner task per update when it receives at
 * least D updates: Opt-D (Sec. 4.2, Algorithm 1) picks D from the histogram
 * of update counts, Opt-D-Cost (Sec. 4.3) also keeps updates below 50,000
 * flops inside the outer task, and the hybrid rule (Sec. 4.4) switches to a
 * sequential supernode loop over multithreaded dense kernels (mt-BLAS) for
 * matrices with wide supernodes.  Threads are OpenMP; the dense kernels are
 * this library's own (no BLAS).
 *
 * Conventions: int status returns (0 ok, -1 invalid input, -2 not positive
 * definite, -3 out of memory); host memory only; 0-based indices; handles
 * created by the library and freed by the caller (NULL is a no-op).
 */
#ifndef TASKCHOL_H
#define TASKCHOL_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum tch_strategy {
    TCH_NONESTED = 0,    /* one task per supernode, no inner tasks (D = infinity) */
    TCH_NESTED = 1,      /* every update an inner task (D = 1) */
    TCH_OPT_D = 2,       /* inner tasks for supernodes with >= D updates, D by Algorithm 1 */
    TCH_OPT_D_COST = 3,  /* as TCH_OPT_D, inner tasks only for updates of >= cost_threshold flops */
    TCH_MT_BLAS = 4,     /* supernodes one after another, each dense kernel on all threads */
    TCH_HYBRID = 5       /* TCH_MT_BLAS or TCH_OPT_D_COST by the rule of Sec. 4.4 */
};

typedef struct tch_plan_s *tch_plan;

/* Statistics of a plan (the update counts C of Sec. 4.2). */
typedef struct tch_stats {
    int64_t n, nsuper, nnz_a_full;   /* order, supernodes, entries of the full symmetric A */
    int64_t updates;                 /* sum of C[s]: (source, target) update pairs */
    int64_t max_updates;             /* maxChildren of Algorithm 1: the largest C[s] */
    int64_t opt_d;                   /* D chosen by Algorithm 1 */
    int64_t split_opt_d;             /* outer tasks split under Opt-D (C[s] >= D) */
    int64_t tasks_nonested, tasks_nested, tasks_opt_d, tasks_opt_d_cost;  /* outer + inner tasks */
    double avg_supernode_cols;       /* n / nsuper */
    double density;                  /* nnz(A) / n^2 */
    int32_t hybrid_choice;           /* TCH_MT_BLAS or TCH_OPT_D_COST */
    double flops;                    /* sum of squared column counts */
} tch_stats;

/* Result of one factorization. */
typedef struct tch_run {
    double seconds;          /* wall time of the numeric factorization */
    int32_t strategy;        /* the strategy run (TCH_HYBRID resolved) */
    int32_t threads;         /* OpenMP threads used */
    int64_t d;               /* the D used (0: not a nesting strategy) */
    int64_t inner_tasks;     /* inner tasks created */
    int64_t bad_column;      /* permuted column of a failed pivot, or -1 */
} tch_run;

/*
 * tch_plan_create -- the supernodal structure of P^T A P, as the GPU
 * library's analysis exports it (spc_symbolic_export: perm, super_ptr,
 * rptr, rows, sparent; the exact column counts for the flop count), plus
 * the lower CSC pattern of A for the assembly:
 *   n, nsuper        order and supernodes
 *   perm[n]          final order, perm[k] = original index of pivot k
 *   super_ptr[nsuper+1], sparent[nsuper]
 *   rptr[nsuper+1], rows[rptr[nsuper]]   row lists R_s (first w_s = cols(s))
 *   colcount[n]      column counts (flops = sum colcount^2)
 *   colptr[n+1], rowidx[nnz]             lower CSC of A (caller order)
 * The panels of a factorization follow the same layout: supernode s is an
 * m_s x w_s column-major block at offset sum_{t<s} m_t w_t.
 */
int tch_plan_create(int64_t n, int32_t nsuper, const int32_t *perm, const int32_t *super_ptr,
                    const int32_t *sparent, const int64_t *rptr, const int32_t *rows, const int32_t *colcount,
                    const int64_t *colptr, const int32_t *rowidx, tch_plan *out);
int tch_plan_stats(tch_plan p, tch_stats *out);
/* The update count C[s] of every supernode (nsuper entries). */
int tch_plan_update_counts(tch_plan p, int32_t *C);

/* Algorithm 1 (Opt-D): D from n, the number of supernodes and their update
 * counts C (nsuper entries); pure function of its inputs. */
int tch_opt_d(int64_t n, int64_t nsuper, const int32_t *C, int64_t *D);

/* The hybrid rule of Sec. 4.4: TCH_MT_BLAS if the average supernode width
 * exceeds 50, or exceeds 20 with a density below 1e-4; else TCH_OPT_D_COST. */
int tch_hybrid_choice(double avg_supernode_cols, double density);

/*
 * tch_factor -- numeric factorization with `strategy` on `threads` OpenMP
 * threads (0: the OpenMP default).  values: A's entries in the caller's CSC
 * order; Lx: receives the panels (strict upper triangles of the diagonal
 * blocks zero).  d_override > 0 replaces Algorithm 1's D (TCH_OPT_D,
 * TCH_OPT_D_COST); cost_threshold <= 0 takes the paper's 50,000 flops.
 * Returns 0 or -2 (run->bad_column set).  run may be NULL.
 */
int tch_factor(tch_plan p, const double *values, double *Lx, int strategy, int threads, int64_t d_override,
               double cost_threshold, tch_run *run);

void tch_plan_free(tch_plan p);

#ifdef __cplusplus
}
#endif
#endif /* TASKCHOL_H */
