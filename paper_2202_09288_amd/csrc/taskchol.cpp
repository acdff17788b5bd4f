// taskchol.cpp -- the paper's task-parallel left-looking supernodal Cholesky
// on the host (include/taskchol.h), the multicore CPU baseline of the GPU
// library.  Outer tasks (one per supernode) follow the elimination tree; an
// outer task may split its updates into inner tasks (selective nesting,
// Sec. 4); mt-BLAS runs the supernodes one after another with each dense
// kernel on all threads.  OpenMP for the threads; dense kernels of its own.
#include <omp.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "../../include/taskchol.h"

namespace {

constexpr int kNb = 64;          // column block of the dense POTRF/TRSM/trailing update
constexpr int kUpdCols = 128;    // update columns computed per buffer
constexpr double kCostDefault = 50000.0;  // Sec. 4.3: inner tasks below this many flops stay inline

// One update pair (source d, target t): rows i0..i1-1 of R_d are columns of
// t; rows i0..m_d-1 of R_d sit at positions rel[rel_off + (r - i0)] of R_t.
struct Pair {
    int32_t d, t, i0, i1;
    int64_t rel_off;
    double cost;  // SYRK m1 (m1 + 1) k + GEMM 2 (m2 - m1) m1 k  (R5)
};

// body(i) for i in [0, count): on the OpenMP threads when par (mt-BLAS),
// else in the calling thread (no parallel region at all).
template <typename Fn>
void for_range(int64_t count, bool par, Fn &&body) {
    if (par && count > 1) {
#pragma omp parallel for schedule(dynamic, 1)
        for (int64_t i = 0; i < count; ++i) body(i);
    } else {
        for (int64_t i = 0; i < count; ++i) body(i);
    }
}

// ---- dense kernels (column-major) ------------------------------------------

// C[M x N] += alpha * A[M x K] B[N x K]^T; register blocks of 8 x 4.
void gemm_nt(int64_t M, int64_t N, int64_t K, double alpha, const double *A, int64_t lda, const double *B,
             int64_t ldb, double *C, int64_t ldc) {
    constexpr int MR = 8, NR = 4, KC = 256;
    for (int64_t k0 = 0; k0 < K; k0 += KC) {
        const int64_t kc = std::min<int64_t>(KC, K - k0);
        for (int64_t j = 0; j < N; j += NR) {
            const int64_t nr = std::min<int64_t>(NR, N - j);
            for (int64_t i = 0; i < M; i += MR) {
                const int64_t mr = std::min<int64_t>(MR, M - i);
                double acc[NR][MR] = {};
                if (mr == MR && nr == NR) {
                    for (int64_t k = 0; k < kc; ++k) {
                        const double *a = A + i + (k0 + k) * lda;
                        const double *b = B + j + (k0 + k) * ldb;
                        for (int jj = 0; jj < NR; ++jj) {
                            const double bv = b[jj];
#pragma omp simd
                            for (int ii = 0; ii < MR; ++ii) acc[jj][ii] += a[ii] * bv;
                        }
                    }
                } else {
                    for (int64_t k = 0; k < kc; ++k) {
                        const double *a = A + i + (k0 + k) * lda;
                        const double *b = B + j + (k0 + k) * ldb;
                        for (int64_t jj = 0; jj < nr; ++jj)
                            for (int64_t ii = 0; ii < mr; ++ii) acc[jj][ii] += a[ii] * b[jj];
                    }
                }
                for (int64_t jj = 0; jj < nr; ++jj)
                    for (int64_t ii = 0; ii < mr; ++ii) C[i + ii + (j + jj) * ldc] += alpha * acc[jj][ii];
            }
        }
    }
}

// Column Cholesky of the jb x jb diagonal block at A (leading dimension
// lda), lower triangle; returns the first failing column or -1.
int64_t potrf_small(int64_t jb, double *A, int64_t lda) {
    for (int64_t j = 0; j < jb; ++j) {
        double *cj = A + j * lda;
        double d = cj[j];
        for (int64_t k = 0; k < j; ++k) d -= A[j + k * lda] * A[j + k * lda];
        if (!(d > 0.0) || !std::isfinite(d)) return j;
        const double ljj = std::sqrt(d);
        cj[j] = ljj;
        for (int64_t i = j + 1; i < jb; ++i) {
            double v = cj[i];
            for (int64_t k = 0; k < j; ++k) v -= A[i + k * lda] * A[j + k * lda];
            cj[i] = v / ljj;
        }
    }
    return -1;
}

// B[M x jb] := B L^{-T}, L the jb x jb lower triangle at Ljj (lda): column
// by column, each column a vector operation over the rows.
void trsm_small(int64_t M, int64_t jb, const double *L, int64_t ldl, double *B, int64_t ldb) {
    for (int64_t c = 0; c < jb; ++c) {
        double *bc = B + c * ldb;
        for (int64_t k = 0; k < c; ++k) {
            const double lck = L[c + k * ldl];
            const double *bk = B + k * ldb;
#pragma omp simd
            for (int64_t r = 0; r < M; ++r) bc[r] -= bk[r] * lck;
        }
        const double inv = 1.0 / L[c + c * ldl];
#pragma omp simd
        for (int64_t r = 0; r < M; ++r) bc[r] *= inv;
    }
}

// POTRF of the w x w diagonal block of an m x w panel and TRSM of its rows
// below (blocked right-looking by kNb columns); `par` spreads the TRSM rows
// and the trailing update's column blocks over the OpenMP threads
// (mt-BLAS).  Returns the first failing column or -1.
int64_t panel_factor(double *P, int64_t m, int64_t w, bool par) {
    for (int64_t j0 = 0; j0 < w; j0 += kNb) {
        const int64_t jb = std::min<int64_t>(kNb, w - j0);
        double *Djj = P + j0 + j0 * m;
        const int64_t bad = potrf_small(jb, Djj, m);
        if (bad >= 0) return j0 + bad;
        const int64_t r0 = j0 + jb, M = m - r0;
        if (M <= 0) continue;
        // TRSM of every row below the block (the rest of the diagonal block
        // and the rows below the supernode)
        const int64_t nchunk = par ? std::max<int64_t>(1, M / 256) : 1;
        for_range(nchunk, par, [&](int64_t q) {
            const int64_t a = r0 + q * M / nchunk, b = r0 + (q + 1) * M / nchunk;
            trsm_small(b - a, jb, Djj, m, P + a + j0 * m, m);
        });
        // trailing update of columns r0..w-1, one kNb column block at a time
        // (rows from the block's first column: the lower part only)
        const int64_t nbk = (w - r0 + kNb - 1) / kNb;
        for_range(nbk, par, [&](int64_t q) {
            const int64_t c0 = r0 + q * kNb, cb = std::min<int64_t>(kNb, w - c0);
            gemm_nt(m - c0, cb, jb, -1.0, P + c0 + j0 * m, m, P + c0 + j0 * m, m, P + c0 + c0 * m, m);
        });
    }
    for (int64_t c = 1; c < w; ++c)
        for (int64_t i = 0; i < c; ++i) P[i + c * m] = 0.0;
    return -1;
}

}  // namespace

struct tch_plan_s {
    int64_t n = 0;
    int32_t ns = 0;
    std::vector<int32_t> super_ptr, sparent, rows, nchild, C;
    std::vector<int64_t> rptr, lptr;
    std::vector<int64_t> aptr, aent, apos;     // per supernode: caller entries and their panel offsets
    std::vector<Pair> pairs;                   // ascending source
    std::vector<int64_t> uptr;                 // per target: its pairs (ascending source)
    std::vector<int32_t> ulist;
    std::vector<int32_t> rel;
    int64_t nnz_full = 0;
    double flops = 0.0;
};

namespace {

int64_t opt_d(int64_t n, int64_t ns, const int32_t *C) {
    // Algorithm 1: the goal is max(1.1 n_super, n / 14) tasks; D comes down
    // from maxChildren + 1 through the histogram T of the update counts
    // until that many tasks exist, D is at most 0.3 maxChildren and at
    // least n_super / 1000 outer tasks are split.  (T has maxChildren + 1
    // entries, so that T[maxChildren] exists.)
    int64_t maxc = 0;
    for (int64_t i = 0; i < ns; ++i) maxc = std::max<int64_t>(maxc, C[i]);
    std::vector<int64_t> T(maxc + 1, 0);
    for (int64_t i = 0; i < ns; ++i) T[C[i]]++;
    const double goal = std::max(1.1 * (double)ns, (double)n / 14.0);
    int64_t D = maxc + 1, outer = 0, tasks = ns;
    while (((double)tasks < goal || (double)D > 0.3 * (double)maxc || (double)outer < (double)ns / 1000.0) && D > 0) {
        --D;
        outer += T[D];
        tasks += D * T[D];
    }
    return D;
}

int hybrid(double avg, double density) {
    if (avg > 50.0) return TCH_MT_BLAS;
    if (avg > 20.0 && density < 1e-4) return TCH_MT_BLAS;
    return TCH_OPT_D_COST;
}

struct Ctx {
    const tch_plan_s *p;
    const double *values;
    double *Lx;
    int strategy;
    int64_t D;
    double thresh;
    bool par;  // mt-BLAS kernels
    std::vector<omp_lock_t> locks;
    std::unique_ptr<std::atomic<int32_t>[]> pending;
    std::vector<char> failed;         // 2: own pivot failed, 1: a descendant did
    std::vector<int64_t> badcol;
    std::atomic<int64_t> inner{0};
};

// Update of pair q into its target's panel: the rows i0.. of R_d times rows
// i0..i1-1, kUpdCols columns at a time through a buffer, subtracted through
// the relative indices; `lock` guards the target panel when inner tasks of
// the same target may run at once.  `par` computes the column blocks on all
// threads (mt-BLAS: each block lands in other target columns).
void apply_update(Ctx &cx, const Pair &q, bool lock) {
    const tch_plan_s &p = *cx.p;
    const int64_t md = p.rptr[q.d + 1] - p.rptr[q.d], wd = p.super_ptr[q.d + 1] - p.super_ptr[q.d];
    const int64_t mt = p.rptr[q.t + 1] - p.rptr[q.t], ft = p.super_ptr[q.t];
    const double *Ld = cx.Lx + p.lptr[q.d];
    double *Pt = cx.Lx + p.lptr[q.t];
    const int32_t *Rd = p.rows.data() + p.rptr[q.d];
    const int32_t *rel = p.rel.data() + q.rel_off;
    const int64_t nblk = (q.i1 - q.i0 + kUpdCols - 1) / kUpdCols;
    const bool par = cx.par && q.cost > 1e6;
    for_range(nblk, par, [&](int64_t b) {
        const int64_t c0 = q.i0 + b * kUpdCols, c1 = std::min<int64_t>(c0 + kUpdCols, q.i1);
        const int64_t M = md - c0, N = c1 - c0;
        thread_local std::vector<double> buf;
        if ((int64_t)buf.size() < M * N) buf.resize(M * N);
        std::fill(buf.begin(), buf.begin() + M * N, 0.0);
        gemm_nt(M, N, wd, 1.0, Ld + c0, md, Ld + c0, md, buf.data(), M);
        if (lock) omp_set_lock(&cx.locks[q.t]);
        for (int64_t c = 0; c < N; ++c) {
            double *col = Pt + (int64_t)(Rd[c0 + c] - ft) * mt;
            const double *u = buf.data() + c * M;
            for (int64_t r = c; r < M; ++r) col[rel[c0 - q.i0 + r]] -= u[r];
        }
        if (lock) omp_unset_lock(&cx.locks[q.t]);
    });
}

// The outer task of supernode s: build, updates (inline or inner tasks),
// POTRF + TRSM; then release its parent when it was the last child.
void outer(Ctx &cx, int32_t s) {
    const tch_plan_s &p = *cx.p;
    const int64_t m = p.rptr[s + 1] - p.rptr[s], w = p.super_ptr[s + 1] - p.super_ptr[s];
    double *P = cx.Lx + p.lptr[s];
    const bool skip = cx.failed[s] != 0;  // a descendant failed: nothing to factor
    if (!skip) {
        std::fill(P, P + m * w, 0.0);
        for (int64_t k = p.aptr[s]; k < p.aptr[s + 1]; ++k) P[p.apos[k]] = cx.values[p.aent[k]];
        const bool nest = (cx.strategy == TCH_NESTED || cx.strategy == TCH_OPT_D || cx.strategy == TCH_OPT_D_COST) &&
                          p.C[s] >= cx.D && p.C[s] > 0;
        Ctx *cxp = &cx;
        for (int64_t u = p.uptr[s]; u < p.uptr[s + 1]; ++u) {
            const Pair *q = &p.pairs[p.ulist[u]];
            if (nest && (cx.strategy != TCH_OPT_D_COST || q->cost >= cx.thresh)) {
                cx.inner++;
#pragma omp task firstprivate(q, cxp)
                apply_update(*cxp, *q, true);
            } else {
                apply_update(cx, *q, nest);
            }
        }
        if (nest) {
#pragma omp taskwait
        }
        const int64_t bad = panel_factor(P, m, w, cx.par);
        if (bad >= 0) {
            cx.failed[s] = 2;
            cx.badcol[s] = p.super_ptr[s] + bad;
        }
    }
    const int32_t par = p.sparent[s];
    if (par >= 0) {
        if (cx.failed[s]) cx.failed[par] = std::max<char>(cx.failed[par], 1);
        // tasks: the last child to finish starts its parent (the loop of
        // mt-BLAS visits supernodes in ascending order instead)
        if (!cx.par && cx.pending[par].fetch_sub(1) == 1) {
            Ctx *cxp = &cx;
#pragma omp task firstprivate(par, cxp)
            outer(*cxp, par);
        }
    }
}

}  // namespace

extern "C" {

int tch_opt_d(int64_t n, int64_t nsuper, const int32_t *C, int64_t *D) {
    if (n < 0 || nsuper < 0 || (nsuper > 0 && !C) || !D) return -1;
    for (int64_t i = 0; i < nsuper; ++i)
        if (C[i] < 0) return -1;
    *D = opt_d(n, nsuper, C);
    return 0;
}

int tch_hybrid_choice(double avg, double density) { return hybrid(avg, density); }

int tch_plan_create(int64_t n, int32_t nsuper, const int32_t *perm, const int32_t *super_ptr,
                    const int32_t *sparent, const int64_t *rptr, const int32_t *rows, const int32_t *colcount,
                    const int64_t *colptr, const int32_t *rowidx, tch_plan *out) {
    if (!out || n < 0 || nsuper < 0 || !perm || !super_ptr || !sparent || !rptr || !rows || !colcount || !colptr ||
        !rowidx)
        return -1;
    *out = nullptr;
    tch_plan_s *p = new (std::nothrow) tch_plan_s;
    if (!p) return -3;
    try {
        p->n = n;
        p->ns = nsuper;
        p->super_ptr.assign(super_ptr, super_ptr + nsuper + 1);
        p->sparent.assign(sparent, sparent + nsuper);
        p->rptr.assign(rptr, rptr + nsuper + 1);
        p->rows.assign(rows, rows + rptr[nsuper]);
        std::vector<int32_t> iperm(n), snode(n);
        for (int64_t k = 0; k < n; ++k) iperm[perm[k]] = (int32_t)k;
        for (int32_t s = 0; s < nsuper; ++s)
            for (int32_t j = super_ptr[s]; j < super_ptr[s + 1]; ++j) snode[j] = s;
        p->lptr.assign(nsuper + 1, 0);
        for (int32_t s = 0; s < nsuper; ++s)
            p->lptr[s + 1] = p->lptr[s] + (rptr[s + 1] - rptr[s]) * (int64_t)(super_ptr[s + 1] - super_ptr[s]);
        for (int64_t j = 0; j < n; ++j) p->flops += (double)colcount[j] * (double)colcount[j];
        // assembly: caller entries grouped by the supernode of their column
        const int64_t nnz = colptr[n];
        std::vector<int32_t> dst(nnz);
        std::vector<int64_t> pos(nnz);
        p->aptr.assign(nsuper + 1, 0);
        for (int64_t c = 0; c < n; ++c)
            for (int64_t k = colptr[c]; k < colptr[c + 1]; ++k) {
                const int32_t a = iperm[rowidx[k]], b = iperm[c];
                const int32_t row = std::max(a, b), col = std::min(a, b), s = snode[col];
                const int32_t *R = rows + rptr[s];
                const int64_t ms = rptr[s + 1] - rptr[s];
                const int32_t *it = std::lower_bound(R, R + ms, row);
                if (it == R + ms || *it != row) {
                    delete p;
                    return -1;
                }
                dst[k] = s;
                pos[k] = (int64_t)(col - super_ptr[s]) * ms + (it - R);
                p->aptr[s + 1]++;
                p->nnz_full += (rowidx[k] == c) ? 1 : 2;
            }
        for (int32_t s = 0; s < nsuper; ++s) p->aptr[s + 1] += p->aptr[s];
        p->aent.resize(nnz);
        p->apos.resize(nnz);
        {
            std::vector<int64_t> fill(p->aptr.begin(), p->aptr.end() - 1);
            for (int64_t k = 0; k < nnz; ++k) {
                const int64_t at = fill[dst[k]]++;
                p->aent[at] = k;
                p->apos[at] = pos[k];
            }
        }
        // update pairs and relative indices
        p->C.assign(nsuper, 0);
        p->nchild.assign(nsuper, 0);
        for (int32_t s = 0; s < nsuper; ++s)
            if (sparent[s] >= 0) p->nchild[sparent[s]]++;
        for (int32_t d = 0; d < nsuper; ++d) {
            const int64_t md = rptr[d + 1] - rptr[d], wd = super_ptr[d + 1] - super_ptr[d];
            const int32_t *Rd = rows + rptr[d];
            int64_t i = wd;
            while (i < md) {
                const int32_t t = snode[Rd[i]];
                int64_t i1 = i;
                while (i1 < md && snode[Rd[i1]] == t) ++i1;
                Pair q;
                q.d = d;
                q.t = t;
                q.i0 = (int32_t)i;
                q.i1 = (int32_t)i1;
                q.rel_off = (int64_t)p->rel.size();
                const int32_t *Rt = rows + rptr[t];
                const int64_t mt = rptr[t + 1] - rptr[t];
                int64_t r = 0;
                for (int64_t k = i; k < md; ++k) {
                    while (r < mt && Rt[r] < Rd[k]) ++r;
                    if (r == mt || Rt[r] != Rd[k]) {
                        delete p;
                        return -1;
                    }
                    p->rel.push_back((int32_t)r);
                }
                const double m1 = (double)(i1 - i), m2 = (double)(md - i), k = (double)wd;
                q.cost = m1 * (m1 + 1.0) * k + 2.0 * (m2 - m1) * m1 * k;
                p->pairs.push_back(q);
                p->C[t]++;
                i = i1;
            }
        }
        p->uptr.assign(nsuper + 1, 0);
        for (const Pair &q : p->pairs) p->uptr[q.t + 1]++;
        for (int32_t s = 0; s < nsuper; ++s) p->uptr[s + 1] += p->uptr[s];
        p->ulist.resize(p->pairs.size());
        {
            std::vector<int64_t> fill(p->uptr.begin(), p->uptr.end() - 1);
            for (size_t k = 0; k < p->pairs.size(); ++k) p->ulist[fill[p->pairs[k].t]++] = (int32_t)k;
        }
    } catch (const std::bad_alloc &) {
        delete p;
        return -3;
    }
    *out = p;
    return 0;
}

int tch_plan_update_counts(tch_plan p, int32_t *C) {
    if (!p || !C) return -1;
    std::copy(p->C.begin(), p->C.end(), C);
    return 0;
}

int tch_plan_stats(tch_plan p, tch_stats *o) {
    if (!p || !o) return -1;
    std::memset(o, 0, sizeof(*o));
    o->n = p->n;
    o->nsuper = p->ns;
    o->nnz_a_full = p->nnz_full;
    o->updates = (int64_t)p->pairs.size();
    for (int32_t c : p->C) o->max_updates = std::max<int64_t>(o->max_updates, c);
    o->opt_d = opt_d(p->n, p->ns, p->C.data());
    o->tasks_nonested = p->ns;
    o->tasks_nested = p->ns + (int64_t)p->pairs.size();
    o->tasks_opt_d = p->ns;
    o->tasks_opt_d_cost = p->ns;
    for (int32_t s = 0; s < p->ns; ++s)
        if (p->C[s] >= o->opt_d && p->C[s] > 0) {
            o->split_opt_d++;
            o->tasks_opt_d += p->C[s];
            for (int64_t u = p->uptr[s]; u < p->uptr[s + 1]; ++u)
                if (p->pairs[p->ulist[u]].cost >= kCostDefault) o->tasks_opt_d_cost++;
        }
    o->avg_supernode_cols = p->ns ? (double)p->n / (double)p->ns : 0.0;
    o->density = p->n ? (double)p->nnz_full / ((double)p->n * (double)p->n) : 0.0;
    o->hybrid_choice = hybrid(o->avg_supernode_cols, o->density);
    o->flops = p->flops;
    return 0;
}

int tch_factor(tch_plan p, const double *values, double *Lx, int strategy, int threads, int64_t d_override,
               double cost_threshold, tch_run *run) {
    if (!p || (!values && p->n > 0) || (!Lx && p->n > 0) || strategy < TCH_NONESTED || strategy > TCH_HYBRID ||
        threads < 0)
        return -1;
    if (strategy == TCH_HYBRID) {
        tch_stats st;
        tch_plan_stats(p, &st);
        strategy = st.hybrid_choice;
    }
    Ctx cx;
    cx.p = p;
    cx.values = values;
    cx.Lx = Lx;
    cx.strategy = strategy;
    cx.thresh = cost_threshold > 0.0 ? cost_threshold : kCostDefault;
    cx.par = strategy == TCH_MT_BLAS;
    cx.D = strategy == TCH_NESTED ? 1
           : (strategy == TCH_OPT_D || strategy == TCH_OPT_D_COST)
               ? (d_override > 0 ? d_override : opt_d(p->n, p->ns, p->C.data()))
               : INT64_MAX;
    const int nt = threads > 0 ? threads : omp_get_max_threads();
    cx.locks.resize(p->ns);
    for (auto &l : cx.locks) omp_init_lock(&l);
    cx.pending.reset(new std::atomic<int32_t>[std::max(1, p->ns)]);
    for (int32_t s = 0; s < p->ns; ++s) cx.pending[s] = p->nchild[s];
    cx.failed.assign(p->ns, 0);
    cx.badcol.assign(p->ns, -1);
    int used = 1;
    const auto t0 = std::chrono::steady_clock::now();
    if (strategy == TCH_MT_BLAS) {
        // supernodes in ascending order (children first), kernels threaded
        omp_set_max_active_levels(1);
        int saved = omp_get_max_threads();
        omp_set_num_threads(nt);
        used = nt;
        for (int32_t s = 0; s < p->ns; ++s) outer(cx, s);
        omp_set_num_threads(saved);
    } else {
#pragma omp parallel num_threads(nt)
        {
#pragma omp single
            {
                used = omp_get_num_threads();
                Ctx *cxp = &cx;
                for (int32_t s = 0; s < p->ns; ++s)
                    if (p->nchild[s] == 0) {
#pragma omp task firstprivate(s, cxp)
                        outer(*cxp, s);
                    }
            }
        }
    }
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (auto &l : cx.locks) omp_destroy_lock(&l);
    int rc = 0;
    int64_t bad = -1;
    for (int32_t s = 0; s < p->ns; ++s)
        if (cx.failed[s] == 2) {
            rc = -2;
            bad = cx.badcol[s];
            break;
        }
    if (run) {
        run->seconds = sec;
        run->strategy = strategy;
        run->threads = used;
        run->d = (strategy == TCH_OPT_D || strategy == TCH_OPT_D_COST || strategy == TCH_NESTED) ? cx.D : 0;
        run->inner_tasks = cx.inner.load();
        run->bad_column = bad;
    }
    return rc;
}

void tch_plan_free(tch_plan p) { delete p; }

}  // extern "C"
