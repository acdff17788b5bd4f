// plan.h -- host-side symbolic analysis and the device schedule built from it.
//
// Internal to the library: nothing here crosses the C ABI.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace spc {

// Tile edges of the update kernels; scatter updates of dimension >=
// kBigMin with a contraction of at least kBigMinK use the large tiles.
constexpr int kTile = 64;
constexpr int kTileBig = 128;
constexpr int kBigMin = 256;
constexpr int kBigMinK = 128;
// Supernodes with w <= kSmallW and m <= kSmallM are factored, inverted and
// scatter-added by one workgroup each (k_small); those with w <= kTinyW and
// m <= kTinyM by one wave each (k_tiny, four per workgroup).
constexpr int kSmallW = 32;
constexpr int kSmallM = 128;
constexpr int kTinyW = 8;
constexpr int kTinyM = 64;
// Tiny supernodes with w <= kGroupW and m <= 16 (32) share a wave, four
// (two) to a wave, 16 (32) lanes each.
constexpr int kGroupW = 4;
// Width of the column blocks a supernode is cut into, for the panel
// factorization and for the triangular solves alike; each block's diagonal
// triangle gets an explicit inverse in the inverse store.
constexpr int kNB = 64;
constexpr int kPanelNB = kNB;
// Column blocks per bulk trailing update (default; a tuning option): the
// columns beyond a group of `delay` blocks are updated once, with all of the
// group's panels (K = delay * kNB), while each next block inside the group
// is brought up to date on its own just before it is factored.  Measured on
// the 60^3 grid: 1 -> 16.3 ms, 2 -> 16.6, 3 -> 17.0, 4 -> 17.3 (the
// column-only launches lengthen the chain of dependent steps more than the
// deeper updates save); workloads whose top supernodes are bound by the
// trailing update's memory traffic rather than by that chain can gain.
constexpr int kDelay = 1;
constexpr int kDelayMax = 8;
constexpr int kSolveNB = kNB;
// Rows of one solve-update task.
constexpr int kSolveRows = 256;
// Solve levels from the top with fewer tasks than this run as one
// persistent launch per sweep; the wide levels below keep one launch each
// (measured on the 60^3 grid: 64 -> 4.2 ms, 256 -> 3.7, 1024 -> 3.55, all
// levels persistent -> 4.9).
constexpr int kSolvePersistMax = 1024;

// Schedule cut-offs of one analysis (the defaults above, or chosen per
// workload through the analysis options, e.g. by the autotuner).  The
// tiny and small limits are bounded by what their kernels hold (kTinyW x
// kTinyM in one wave, kSmallW x kSmallM in one workgroup's LDS); 0 turns a
// path off.
struct Tuning {
    int32_t tiny_w = kTinyW, tiny_m = kTinyM;
    int32_t small_w = kSmallW, small_m = kSmallM;
    int32_t big_min = kBigMin, big_min_k = kBigMinK;
    int32_t solve_persist_max = kSolvePersistMax;
    int32_t handover = 1;  // fused TRSM with in-launch waits (0: off, 2: only where few tiles wait)
    int32_t delay = kDelay;  // column blocks per bulk trailing update
    int32_t persist = 0;     // small subtrees in one persistent launch (0: per level)
    int32_t ordering = 0;    // order computed by analyze when none is given (order_graph's method)
    int32_t group = 1;       // tiny supernodes of 16 / 32 rows share a wave (0: one wave each)
    int32_t bulk128 = 0;     // bulk trailing updates (K >= 128) on 128x128 tiles in a launch of their own
    int32_t lookahead = 0;   // bulk update beyond the next group spread over that group's steps (delay >= 2)
};

// One pair (source supernode s, ancestor t) of the scatter: rows
// i0..i1-1 of R_s (positions, i0 >= w_s) are columns of t, and rows
// i0..m_s-1 of R_s sit at positions rel[rel_off + (i - i0)] of R_t.
struct UpdatePair {
    int32_t target;
    int32_t i0;
    int32_t i1;
    int32_t pad;
    int64_t rel_off;
};

// One output tile of a SYRK/GEMM update of supernode s: rows i0..i0+63 and
// columns j0..j0+63 (positions in R_s) of P P^T with P the columns
// k0..k1-1 of the panel.  A TRSM tile is rows i0..i0+63 of block `blk`
// (columns k0..k1-1) multiplied by the transposed block inverse.  Every
// task carries the offsets its kernel needs, so a launch reads its task
// and then the data, with no further dependent lookups.
struct TileTask {
    int64_t loff;   // lptr[s]: the m x w panel
    int64_t aux;    // scatter tiles: rptr[s] (row list); TRSM tiles: inv_off
                    // of the block; the next block's diagonal tile: inv_off
                    // of that block, which its workgroup factors
    int32_t s;
    int32_t m;      // rows of the panel (leading dimension)
    int32_t i0;
    int32_t j0;
    int32_t k0;
    int32_t k1;
    int32_t jmax;   // columns j >= jmax are outside the update
    int32_t blk;    // TRSM tiles: block id.  Trailing tiles: -1, or, for the
                    // tiles of the next column block's columns (j0 = k1),
                    // that block's global first column: the diagonal tile's
                    // workgroup (i0 = j0) factors the block after updating it
    int32_t flag;   // trailing tiles of the next block's columns, when that
                    // block is a full kNB wide: its block id q, which owns
                    // the hand-over words 5q..5q+4 (one flag per 16-column
                    // panel, then the claim of the block's factorization).
                    // The workgroup that claims it (the diagonal tile's, or
                    // the first tile below to arrive) hands out each panel
                    // (its L and the inverse of its diagonal triangle,
                    // inside the inverse at aux) as soon as it is factored;
                    // each tile below follows panel by panel with the
                    // block's TRSM on its own rows.  -1 otherwise.
    int32_t pad;
};

// POTRF of the block of columns c0..c1-1 (c0 a multiple of kNB) of
// supernode s: factor the diagonal triangle and write its inverse at ioff.
struct PanelTask {
    int64_t loff;  // lptr[s]
    int64_t ioff;  // inv_off[blk]
    int32_t s;
    int32_t m;
    int32_t c0;
    int32_t c1;
    int32_t g0;    // global column of c0 (pivot reports)
    int32_t pad;
};

// A whole small supernode (k_small): factor, invert, scatter its update.
struct SmallTask {
    int64_t loff;  // lptr[s]
    int64_t roff;  // rptr[s]
    int64_t ioff;  // inv_off of its single block
    int32_t s;
    int32_t m;
    int32_t w;
    int32_t g0;    // global column of its first column
};

// One entry of the persistent launch over the small subtrees: one small
// supernode (kind 0, psmall[first]) or tiny ones, ptiny[first .. first +
// count - 1]: up to four, one wave each (kind 1), up to 16 in groups of 16
// lanes (kind 2), up to 8 in groups of 32 lanes (kind 3).
struct PersistEntry {
    int32_t kind;
    int32_t first;
    int32_t count;
    int32_t pad;
};

// One column block of a supernode (solves and inverse store).
struct SolveBlock {
    int32_t s;
    int32_t c0;      // first column (position in the panel)
    int32_t c1;      // one past the last column
    int32_t ntasks;  // solve-update tasks of this block (>= 1)
};

// Rows r0..r1-1 (positions in R_s, r0 >= c1) below one column block.
struct SolveTask {
    int64_t loff;    // lptr[s]
    int64_t roff;    // rptr[s]
    int64_t ioff;    // inv_off[blk]
    int64_t g0;      // global (permuted) index of the block's first column
    int32_t m;
    int32_t c0;
    int32_t nb;      // block width
    int32_t r0;
    int32_t r1;
    int32_t ntasks;  // tasks of the block
    int32_t blk;
    int32_t first;   // 1 for the block's first task
    // Persistent sweeps, hand-over between blocks q - 1 and q of one
    // supernode: bit 0 on every task of q (forward: the sums of q - 1's
    // first task for q's rows come through the hand-over buffer; backward,
    // on q's first task: x_q goes out through it too); bit 1 on the first
    // task of q - 1, whose first (hand >> 8) rows are q's (forward: their
    // sums go out through the buffer; backward: their x come in through it).
    int32_t hand;
    int32_t pad;
};
constexpr int32_t kHandIn = 1, kHandOut = 2;

struct Symbolic {
    Tuning tune;
    int64_t n = 0, nnzA = 0;
    std::vector<int32_t> perm, iperm, parent, colcount;
    int32_t nsuper = 0;
    std::vector<int32_t> super_ptr, snode, sparent, level;
    std::vector<int64_t> rptr, lptr;
    std::vector<int32_t> rows;
    int64_t flops = 0, nnzL = 0, max_w = 0, max_m = 0;
    int32_t nlevels = 0;
    std::vector<int64_t> amap;  // caller entry k -> panel offset
    std::vector<int64_t> dsrc;  // permuted column j -> caller entry of its diagonal
    // full symmetric A in the caller's ordering (CSR), entries pointing into
    // the caller's lower-CSC values; used by iterative refinement
    std::vector<int64_t> csr_ptr, csr_val;
    std::vector<int32_t> csr_col;

    // scatter plan
    std::vector<int64_t> pair_ptr;     // [nsuper+1] pairs of each source
    std::vector<UpdatePair> pairs;
    std::vector<int32_t> colpair;      // [rows_total] pair of each below row
    std::vector<int32_t> rel;

    // factor schedule: for each level, a list of steps; each step is a
    // panel-task range followed by a tile-task range
    // Step b of a level: POTRF of block 0 (b = 0 only), TRSM of block b,
    // then the trailing update by panel b, split in two: the tiles of block
    // b+1's own columns (t0..tm, which also factor block b+1) and the tiles
    // of the columns beyond (tm..t1), which can run beside the next step's
    // TRSM and column update (lookahead).
    struct Step {
        int64_t f0, f1;   // POTRF tasks
        int64_t p0, p1;   // TRSM tiles
        int64_t t0, tm, t1;  // trailing tiles: next block's columns, then the rest
        int64_t q0, q1;      // bulk trailing tiles on 128x128 (trail_big), a launch after the trailing one
        double potrf_flops, trsm_flops, look_flops, rest_flops, big_flops;  // algorithmic flops of its launches
    };
    std::vector<int64_t> level_step_ptr;   // [nlevels+1]
    std::vector<Step> steps;
    std::vector<int64_t> ext_tile_ptr;     // [nlevels+1] external tiles (64)
    std::vector<int64_t> ext_big_ptr;      // [nlevels+1] external tiles (128)
    std::vector<TileTask> trail_big;       // bulk trailing tiles (128), by step
    std::vector<int64_t> small_ptr;        // [nlevels+1] into small_tasks
    std::vector<SmallTask> small_tasks;    // supernodes of the single-workgroup path
    std::vector<int64_t> tiny_ptr;         // [nlevels+1] into tiny_tasks
    std::vector<SmallTask> tiny_tasks;     // supernodes of the single-wave path
    // per level, tiny_tasks[tiny_ptr[l] .. tiny_e16[l]) go in groups of 16
    // lanes, [tiny_e16[l] .. tiny_e32[l]) in groups of 32, the rest one wave each
    std::vector<int64_t> tiny_e16, tiny_e32;  // [nlevels]
    // Scatter addressing per row position k >= w_s of R_s (pair p of k,
    // target t): cbase = lptr[t] + (rows[k] - first column of t) * m_t is
    // column rows[k] of t's panel; crel = rel_off(p) - i0(p), so row
    // position i >= k of R_s lands at cbase + rel[crel + i].
    std::vector<int64_t> cbase, crel;
    std::vector<int32_t> first_blk;        // [nsuper+1] first column block
    std::vector<double> small_flops;       // [nlevels] flops of the small path
    std::vector<double> tiny_flops;        // [nlevels] flops of the single-wave path
    std::vector<double> ext_flops;         // [nlevels] flops of the 64-tile scatter launch
    std::vector<double> ext_big_flops;     // [nlevels] flops of the 128-tile scatter launch
    // Persistent launch over every small subtree (a supernode whose whole
    // subtree is small or tiny), all levels at once: queue entries in level
    // order; a supernode waits until the scatters of every source inside
    // that set into it have counted pdep0[s] down to zero, and after its own
    // scatter counts down the targets ptgt[ptgt_ptr[s] ..] inside the set.
    std::vector<SmallTask> psmall, ptiny;
    std::vector<PersistEntry> pqueue;
    // chunks of consecutive queue entries of one level, taken by one
    // workgroup per work-counter increment (up to 16 entries where the level
    // is wide, so that the counter is not contended): [nchunks+1]
    std::vector<int32_t> pchunk;
    std::vector<int32_t> pdep0;            // [nsuper]
    std::vector<int64_t> ptgt_ptr;         // [nsuper+1]
    std::vector<int32_t> ptgt;
    double persist_flops = 0.0;
    std::vector<PanelTask> potrf_tasks;
    std::vector<TileTask> trsm_tiles;
    std::vector<TileTask> int_tiles;
    std::vector<TileTask> ext_tiles;
    std::vector<TileTask> ext_tiles_big;

    // column blocks, their inverse-store offsets, and the solve schedule
    // (blocks grouped by block-tree level)
    std::vector<SolveBlock> sblocks;
    std::vector<int64_t> inv_off;          // [nblocks+1]
    std::vector<int64_t> slevel_ptr;       // [nslevels+1] into sblock_order
    std::vector<int32_t> sblock_order;
    std::vector<int64_t> stask_ptr;        // [nslevels+1] into stasks
    std::vector<SolveTask> stasks;
    std::vector<int64_t> stiny_ptr;        // [nslevels+1] into stiny
    std::vector<SmallTask> stiny;          // tiny supernodes of levels < solve_split (one wave each)
    int32_t nslevels = 0;
    // Persistent solves: for each task the column blocks its rows fall in
    // (ascending, distinct), for each block the number of (task, block)
    // contributions its forward step waits for, and the task order of the
    // backward sweep (block-tree levels from the top).
    // Levels solve_split.. run persistently; fdep counts only their tasks,
    // and bwd_order lists only their tasks.
    int32_t solve_split = 0;
    std::vector<int64_t> stgt_ptr;
    std::vector<int32_t> stgt;
    std::vector<int32_t> fdep;
    std::vector<int32_t> bwd_order;

    // batches: status word of each supernode (empty: one word)
    std::vector<int32_t> status_slot;

    int64_t rows_total() const { return rptr.empty() ? 0 : rptr.back(); }
    int64_t panel_entries() const { return lptr.empty() ? 0 : lptr.back(); }
};

// A fill-reducing order of a lower-CSC pattern (perm[k] = vertex eliminated
// k-th): method 0 the identity, 1 graph nested dissection by level
// structures, 2 minimum degree (n <= 10,000).  0, or -1 for invalid input.
int order_graph(int64_t n, const int64_t *colptr, const int32_t *rowidx, int method, int32_t *perm);

// Returns 0 or a negative spc_status.
int analyze(int64_t n, const int64_t *colptr, const int32_t *rowidx, const int32_t *perm,
            double z, const Tuning &tune, Symbolic &S);
// Schedule of an analysis whose structural arrays are set.
int build_schedule(Symbolic &S);
// Host check of a schedule's invariants: every block of the blocked path
// has the rows below it solved exactly once (TRSM launch or hand-over
// tiles), and every tile that waits inside a trailing launch comes after its
// diagonal tile and carries the task that tile runs (which it runs itself
// when it claims the block's factorization).  0, or -1 with msg.
int verify_schedule(const Symbolic &S, std::string &msg);
// Disjoint union of analyses with a schedule over the whole forest; the
// offsets of each part (columns, panel entries, inverse store, caller
// entries) are returned, with a final total.
int merge(const std::vector<const Symbolic *> &parts, Symbolic &M, std::vector<int64_t> &col_off,
          std::vector<int64_t> &panel_off, std::vector<int64_t> &inv_base, std::vector<int64_t> &val_off);

}  // namespace spc
