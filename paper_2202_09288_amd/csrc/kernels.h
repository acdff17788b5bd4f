// kernels.h -- host-side launchers of the device kernels (internal).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace spc {

// Device copy of the symbolic arrays and task lists the kernels read.
struct DevPlan {
    const int32_t *rows;        // row lists R_s (solves)
    const int32_t *rel;         // relative indices of the scatter pairs
    const int64_t *cbase;       // per row position: target column base
    const int64_t *crel;        // per row position: offset into rel
    const int64_t *amap;        // caller entry -> panel entry
    const int32_t *perm;
    const int64_t *dsrc;        // permuted column -> caller entry of its diagonal
    const PanelTask *potrf_tasks;
    const SmallTask *small_tasks;
    const SmallTask *tiny_tasks;
    const TileTask *trsm_tiles;
    const TileTask *int_tiles;
    const TileTask *ext_tiles;
    const TileTask *ext_tiles_big;
    const TileTask *trail_big;   // bulk trailing updates on 128x128 tiles
    const SolveTask *stasks;
    const SmallTask *stiny;      // one-wave solve tasks (tiny supernodes)
    const int32_t *status_slot;  // supernode -> status word, or null (one word)
    const int64_t *stgt_ptr;     // persistent solves: target blocks per task
    const int32_t *stgt;
    const int32_t *fdep;         // forward contributions per block
    const int32_t *bwd_order;    // task order of the backward sweep
    const PersistEntry *pqueue;  // persistent launch over the small subtrees
    const int32_t *pchunk;
    const SmallTask *psmall;
    const SmallTask *ptiny;
    const int32_t *pdep0;
    const int64_t *ptgt_ptr;
    const int32_t *ptgt;
};

// Bounded waits on other workgroups: `err` is the factor's device-error
// word (set when a wait gives up, cleared by a factorization), `spin` the
// polls before a wait gives up.
struct WaitCtl {
    int32_t *err;
    int32_t spin;
};
// Pivot floors of a factorization with BF16 updates: a pivot below v[g]
// (global permuted column g; v = theta * the column's diagonal entry of A)
// is raised to v[g], and *count counts them.  v == nullptr: off.
template <typename T>
struct PivotFloor {
    const T *v = nullptr;
    int32_t *count = nullptr;
};
// theta: the unit roundoff of BF16 (8 significant bits), 2^-8.
constexpr double kBf16PivotTheta = 1.0 / 256.0;

// Hand-over words per 64-column block: the flags of its four 16-column
// panels, then the claim of its factorization.
constexpr int kFlagsPerBlock = 5;
// Polls of a bounded wait by default: about a second.
constexpr int32_t kSpinDefault = 1 << 20;

// Device state of one persistent solve (in the caller's workspace):
// kSolveSyncInts(nblocks) int32 words, plus the factor's error word.
struct SolveSync {
    int32_t *dep;    // [nblocks] forward contributions still due
    int32_t *done;   // [nblocks] 1 once x of the block is final (backward)
    int32_t *cnt;    // [nblocks] backward tasks of the block that arrived
    int32_t *queue;  // [2] work counters of the two sweeps
    int32_t *err;    // the factor's device-error word: nonzero once a wait gave up
    int32_t spin;    // polls before a wait gives up
};
inline int64_t kSolveSyncInts(int64_t nblocks) { return 3 * nblocks + 2; }
inline SolveSync make_solve_sync(int32_t *base, int64_t nblocks, WaitCtl wc) {
    return SolveSync{base, base + nblocks, base + 2 * nblocks, base + 3 * nblocks, wc.err, wc.spin};
}

enum { kTilesTrailing = 0, kTilesScatter = 1, kTilesTrsm = 2 };

// Bytes of the per-device scratch array that spc_solve_noalloc works in.
constexpr size_t kScratchBytes = size_t(64) << 20;
// Device address of the scratch array on `device` (looked up once per device,
// with that device current; the array's name in host code is only a stand-in
// for the symbol).  SPC_OK or SPC_DEVICE_ERROR.
int scratch_address(int device, void **out);

// status word: lowest permuted column whose pivot failed, or ~0ull; the
// device-error word and the hand-over flags of the trailing launches (one
// per 16-column panel of each column block) to 0
void launch_status_reset(unsigned long long *status, int count, int32_t *deverr, int32_t *flags, int nflags,
                         hipStream_t st);
template <typename T>
void launch_zero(T *x, int64_t count, hipStream_t st);
template <typename T>
void launch_assemble(const DevPlan &P, int64_t nnz, const double *values, T *Lx, hipStream_t st);
// floor[j] = theta * A's diagonal entry of permuted column j (BF16 updates)
template <typename T>
void launch_pivot_floor(const DevPlan &P, int64_t n, const double *values, double theta, T *floor, hipStream_t st);
template <typename T>
void launch_potrf(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, T *Linv, unsigned long long *status,
                  int32_t *deverr, PivotFloor<T> pfl, hipStream_t st);
template <typename T>
void launch_small(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, T *Linv, unsigned long long *status,
                  PivotFloor<T> pfl, hipStream_t st);
template <typename T>
// tasks t0..t16-1 in groups of 16 lanes, t16..t32-1 in groups of 32, the
// rest one wave each
void launch_tiny(const DevPlan &P, int64_t t0, int64_t t16, int64_t t32, int64_t t1, T *Lx, T *Linv,
                 unsigned long long *status, PivotFloor<T> pfl, hipStream_t st);
template <typename T>
// bf16: (float panels only) the trailing and scatter updates multiply
// operands rounded to BF16 on BF16 MFMA with FP32 accumulation
void launch_tiles(const DevPlan &P, int mode, int64_t t0, int64_t t1, T *Lx, T *Linv, unsigned long long *status,
                  int32_t *hflags, WaitCtl wc, bool bf16, PivotFloor<T> pfl, hipStream_t st);

template <typename T>
void launch_tiles128(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, bool bf16, hipStream_t st);
// The bulk trailing updates trail_big[t0..t1) on 128x128 tiles (in place).
template <typename T>
void launch_trail128(const DevPlan &P, int64_t t0, int64_t t1, T *Lx, bool bf16, hipStream_t st);

// The persistent launch over the small subtrees (nchunks chunks of queue
// entries, nsuper dependency counters in pdep, one work counter): resets the
// counters, then runs every entry.
template <typename T>
void launch_persist_small(const DevPlan &P, int64_t nchunks, int64_t nsuper, int32_t *pdep, int32_t *qctr, T *Lx,
                          T *Linv, unsigned long long *status, PivotFloor<T> pfl, WaitCtl wc, hipStream_t st);

template <typename T>
void launch_perm_in(const DevPlan &P, int64_t n, int nrhs, const double *B, int64_t ldb, T *W,
                    hipStream_t st);
template <typename T>
void launch_perm_out(const DevPlan &P, int64_t n, int nrhs, const T *W, double *B, int64_t ldb,
                     hipStream_t st);
void launch_solve_reset(const DevPlan &P, int64_t nblocks, SolveSync sy, hipStream_t st);
// Solve sweeps over tasks t0..t1-1 (one block-tree level), or, with
// persist, over the tasks of levels solve_split.. in one persistent launch
// (t0 = first task of that range, t1 = all tasks; needs launch_solve_reset
// first).
// H (forward) and XB (backward): the persistent sweeps' hand-over buffers,
// n x nrhs like Y, every entry unset (launch_fill_unset) before the sweep.
template <typename T>
void launch_solve_fwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *Y, T *X, T *H,
                      int64_t n, int nrhs, SolveSync sy, bool persist, hipStream_t st);
// One-wave solve sweeps over the tiny supernodes t0..t1-1 of one level.
template <typename T>
void launch_solve_tiny_fwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *Y, T *X,
                           int64_t n, int nrhs, hipStream_t st);
template <typename T>
void launch_solve_tiny_bwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *X, int64_t n,
                           int nrhs, hipStream_t st);
template <typename T>
void launch_solve_bwd(const DevPlan &P, int64_t t0, int64_t t1, const T *Lx, const T *Linv, T *X, T *Acc, T *XB,
                      int64_t n, int nrhs, SolveSync sy, bool persist, hipStream_t st);
template <typename T>
void launch_fill_unset(T *p, int64_t count, hipStream_t st);

// refinement (FP64)
void launch_spmv(const int64_t *rowptr, const int32_t *colidx, const int64_t *valmap, const double *values,
                 const double *X, const double *B, double *Y, int64_t n, int64_t nnz, int nrhs, int64_t ld,
                 hipStream_t st);
void launch_norm_inf_A(const int64_t *rowptr, const int64_t *valmap, const double *values, int64_t n, int64_t nnz,
                       unsigned long long *out, hipStream_t st);
void launch_colmax(const double *V, int64_t n, int nrhs, int64_t ld, unsigned long long *out, hipStream_t st);
void launch_coldot(const double *U, const double *V, int64_t n, int nrhs, int64_t ld, double *out, hipStream_t st);
// The conjugate-gradient coefficients of K slots on the device (alpha, or
// beta with the update of rho); frozen[j] != 0 marks a converged slot.
void launch_cg_coef(const double *dots, double *rho, const double *frozen, double *coef, int64_t K, bool alpha,
                    hipStream_t st);
void launch_axpby(const double *a, double a0, const double *X, const double *b, double b0, double *Y, int64_t n,
                  int nrhs, int64_t ld, hipStream_t st);
void launch_copy_cols(const double *X, int64_t ldx, double *Y, int64_t ldy, int64_t n, int nrhs, hipStream_t st);
// segmented forms (batches): row i belongs to system seg[i]; results and
// coefficients per (column q, system) at q * nseg + seg[i]; norm_inf_A per
// system
void launch_seg_norm_inf_A(const int64_t *rowptr, const int64_t *valmap, const double *values, const int32_t *seg,
                           int64_t n, unsigned long long *out, hipStream_t st);
void launch_seg_colmax(const double *V, const int32_t *seg, int64_t n, int nrhs, int64_t ld, int nseg,
                       unsigned long long *out, hipStream_t st);
void launch_seg_coldot(const double *U, const double *V, const int32_t *seg, int64_t n, int nrhs, int64_t ld,
                       int nseg, double *out, hipStream_t st);
void launch_seg_axpby(const double *a, double a0, const double *X, const double *b, double b0, double *Y,
                      const int32_t *seg, int64_t n, int nrhs, int64_t ld, int nseg, hipStream_t st);
void launch_batch_move(double *const *ptrs, const int64_t *lds, const int64_t *offs, double *M, int64_t n,
                       int count, int nrhs, bool to_merged, hipStream_t st);

}  // namespace spc
