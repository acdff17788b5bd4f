// symbolic.cpp -- host analysis: ordering, elimination tree, column counts,
// supernodes, relative indices and the level schedule of the device kernels.
//
// The analyze phase of a supernodal direct solver (paper Sec. 2, "Background
// on CHOLMOD": reordering, elimination tree setup, node amalgamation).  The
// algorithms here are the classical ones:
//   - elimination tree: Liu's algorithm with path compression over the rows
//     of the lower triangle (J. W. H. Liu, "The role of elimination trees in
//     sparse factorization", SIMAX 1990);
//   - column counts and row lists: traversal of the row subtrees; row i of L
//     is the set of nodes on the tree paths from each j with A_ij != 0 up to
//     i, so every visited node gains row i;
//   - supernodes: fundamental supernodes, then chain amalgamation.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "plan.h"
#include "../../include/spchol.h"

namespace spc {
namespace {

// Strictly-lower pattern of A(p, p) by rows: row i lists columns j < i.
void lower_rows(int64_t n, const int64_t *colptr, const int32_t *rowidx, const int32_t *iperm,
                std::vector<int64_t> &rp, std::vector<int32_t> &ri) {
    rp.assign(n + 1, 0);
    for (int64_t c = 0; c < n; ++c)
        for (int64_t k = colptr[c] + 1; k < colptr[c + 1]; ++k) {
            int32_t a = iperm[rowidx[k]], b = iperm[c];
            rp[std::max(a, b) + 1]++;
        }
    for (int64_t i = 0; i < n; ++i) rp[i + 1] += rp[i];
    ri.resize(rp[n]);
    std::vector<int64_t> cur(rp.begin(), rp.end() - 1);
    for (int64_t c = 0; c < n; ++c)
        for (int64_t k = colptr[c] + 1; k < colptr[c + 1]; ++k) {
            int32_t a = iperm[rowidx[k]], b = iperm[c];
            ri[cur[std::max(a, b)]++] = std::min(a, b);
        }
}

void etree_liu(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &ri,
               std::vector<int32_t> &parent) {
    parent.assign(n, -1);
    std::vector<int32_t> anc(n, -1);
    for (int64_t k = 0; k < n; ++k)
        for (int64_t e = rp[k]; e < rp[k + 1]; ++e) {
            int32_t r = ri[e];
            while (r != -1 && r != k) {
                int32_t next = anc[r];
                anc[r] = (int32_t)k;
                if (next == -1) parent[r] = (int32_t)k;
                r = next;
            }
        }
}

// Postorder with roots and children in ascending order, numbered on exit.
void postorder(int64_t n, const std::vector<int32_t> &parent, std::vector<int32_t> &post) {
    std::vector<int64_t> cptr(n + 2, 0);
    for (int64_t j = 0; j < n; ++j) cptr[(parent[j] == -1 ? n : parent[j]) + 1]++;
    for (int64_t j = 0; j <= n; ++j) cptr[j + 1] += cptr[j];
    std::vector<int32_t> kids(n);
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t j = 0; j < n; ++j) kids[fill[parent[j] == -1 ? n : parent[j]]++] = (int32_t)j;
    // node n is a virtual root over the forest
    post.resize(n);
    std::vector<std::pair<int32_t, int64_t>> st;
    st.reserve(64);
    st.push_back({(int32_t)n, cptr[n]});
    int64_t k = 0;
    while (!st.empty()) {
        auto &top = st.back();
        if (top.second < cptr[top.first + 1]) {
            int32_t c = kids[top.second++];
            st.push_back({c, cptr[c]});
        } else {
            if (top.first != n) post[k++] = top.first;
            st.pop_back();
        }
    }
}

int64_t find_pos(const int32_t *R, int64_t m, int32_t row) {
    const int32_t *p = std::lower_bound(R, R + m, row);
    return (p != R + m && *p == row) ? (p - R) : -1;
}

}  // namespace

int build_schedule(Symbolic &S);

int analyze(int64_t n, const int64_t *colptr, const int32_t *rowidx, const int32_t *perm_in,
            double z, const Tuning &tune, Symbolic &S) {
    // ---- validation --------------------------------------------------------
    if (n < 0 || n > INT32_MAX - 1 || !colptr) return SPC_INVALID_INPUT;
    if (colptr[0] != 0) return SPC_INVALID_INPUT;
    for (int64_t c = 0; c < n; ++c) {
        if (colptr[c + 1] <= colptr[c]) return SPC_INVALID_INPUT;  // diagonal missing
        if (!rowidx) return SPC_INVALID_INPUT;
        if (rowidx[colptr[c]] != c) return SPC_INVALID_INPUT;
        for (int64_t k = colptr[c] + 1; k < colptr[c + 1]; ++k)
            if (rowidx[k] <= rowidx[k - 1] || rowidx[k] >= n) return SPC_INVALID_INPUT;
    }
    S = Symbolic();
    S.tune = tune;
    S.n = n;
    S.nnzA = colptr[n];
    std::vector<int32_t> perm0(n), iperm0(n, -1);
    for (int64_t k = 0; k < n; ++k) {
        int32_t p = perm_in ? perm_in[k] : (int32_t)k;
        if (p < 0 || p >= n || iperm0[p] != -1) return SPC_INVALID_INPUT;
        perm0[k] = p;
        iperm0[p] = (int32_t)k;
    }

    // ---- elimination tree, postorder, final order --------------------------
    std::vector<int64_t> rp;
    std::vector<int32_t> ri, parent0, post;
    lower_rows(n, colptr, rowidx, iperm0.data(), rp, ri);
    etree_liu(n, rp, ri, parent0);
    postorder(n, parent0, post);
    std::vector<int32_t> ipost(n);
    for (int64_t k = 0; k < n; ++k) ipost[post[k]] = (int32_t)k;
    S.perm.resize(n);
    S.iperm.resize(n);
    S.parent.resize(n);
    for (int64_t k = 0; k < n; ++k) {
        S.perm[k] = perm0[post[k]];
        int32_t p = parent0[post[k]];
        S.parent[k] = p == -1 ? -1 : ipost[p];
    }
    for (int64_t k = 0; k < n; ++k) S.iperm[S.perm[k]] = (int32_t)k;
    lower_rows(n, colptr, rowidx, S.iperm.data(), rp, ri);

    // ---- column counts by row subtrees ------------------------------------
    std::vector<int32_t> mark(n, -1);
    std::vector<int64_t> cnt(n, 1);
    for (int64_t i = 0; i < n; ++i) {
        mark[i] = (int32_t)i;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            for (int32_t p = ri[e]; mark[p] != i; p = S.parent[p]) {
                mark[p] = (int32_t)i;
                cnt[p]++;
            }
    }
    S.colcount.resize(n);
    for (int64_t j = 0; j < n; ++j) {
        S.colcount[j] = (int32_t)cnt[j];
        S.nnzL += cnt[j];
        S.flops += cnt[j] * cnt[j];
    }

    // ---- fundamental supernodes -------------------------------------------
    std::vector<int32_t> nkids(n, 0);
    for (int64_t j = 0; j < n; ++j)
        if (S.parent[j] != -1) nkids[S.parent[j]]++;
    std::vector<int32_t> fstart;  // first column of each fundamental supernode
    for (int64_t j = 0; j < n; ++j) {
        bool joins = j > 0 && S.parent[j - 1] == j && nkids[j] == 1 &&
                     S.colcount[j - 1] == S.colcount[j] + 1;
        if (!joins) fstart.push_back((int32_t)j);
    }
    int32_t nf = (int32_t)fstart.size();
    fstart.push_back((int32_t)n);
    std::vector<int32_t> fof(n);
    for (int32_t p = 0; p < nf; ++p)
        for (int32_t j = fstart[p]; j < fstart[p + 1]; ++j) fof[j] = p;

    // ---- chain amalgamation -------------------------------------------------
    // p joins the running group G (which ends in p-1) when p-1's parent
    // supernode is p and the merged group keeps explicit zeros within z of
    // its stored lower-trapezoid entries:
    //   W' = W + w, M' = W + m, Z' = Z + W (M' - M), E' = W'M' - W'(W'-1)/2,
    //   accept iff (double)Z' <= z * (double)E'.
    S.super_ptr.clear();
    int64_t W = 0, M = 0, Z = 0;
    for (int32_t p = 0; p < nf; ++p) {
        int64_t w = fstart[p + 1] - fstart[p];
        int64_t m = S.colcount[fstart[p]];
        bool accept = false;
        if (p > 0) {
            int32_t lastcol = fstart[p] - 1;  // last column of p-1
            int32_t par = S.parent[lastcol];
            if (par != -1 && fof[par] == p) {
                int64_t W2 = W + w, M2 = W + m, Z2 = Z + W * (M2 - M);
                int64_t E2 = W2 * M2 - W2 * (W2 - 1) / 2;
                if ((double)Z2 <= z * (double)E2) {
                    accept = true;
                    W = W2; M = M2; Z = Z2;
                }
            }
        }
        if (!accept) {
            S.super_ptr.push_back(fstart[p]);
            W = w; M = m; Z = 0;
        }
    }
    S.nsuper = (int32_t)S.super_ptr.size();
    S.super_ptr.push_back((int32_t)n);
    const int32_t ns = S.nsuper;
    S.snode.resize(n);
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t j = S.super_ptr[s]; j < S.super_ptr[s + 1]; ++j) S.snode[j] = s;
    S.sparent.resize(ns);
    for (int32_t s = 0; s < ns; ++s) {
        int32_t p = S.parent[S.super_ptr[s + 1] - 1];
        S.sparent[s] = p == -1 ? -1 : S.snode[p];
    }

    // ---- row lists: R_s = cols(s) U (struct(L_{l_s}) below l_s) ----------
    // Every row i > l_s of L in a column of s is also in column l_s (the
    // columns of s are descendants of l_s), so the last column suffices.
    std::vector<int64_t> below(ns, 0);
    std::vector<char> islast(n, 0);
    for (int32_t s = 0; s < ns; ++s) islast[S.super_ptr[s + 1] - 1] = 1;
    std::fill(mark.begin(), mark.end(), -1);
    for (int64_t i = 0; i < n; ++i) {
        mark[i] = (int32_t)i;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            for (int32_t p = ri[e]; mark[p] != i; p = S.parent[p]) {
                mark[p] = (int32_t)i;
                if (islast[p]) below[S.snode[p]]++;
            }
    }
    S.rptr.assign(ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s)
        S.rptr[s + 1] = S.rptr[s] + (S.super_ptr[s + 1] - S.super_ptr[s]) + below[s];
    S.rows.resize(S.rptr[ns]);
    std::vector<int64_t> cur(ns);
    for (int32_t s = 0; s < ns; ++s) {
        int64_t o = S.rptr[s];
        for (int32_t j = S.super_ptr[s]; j < S.super_ptr[s + 1]; ++j) S.rows[o++] = j;
        cur[s] = o;
    }
    std::fill(mark.begin(), mark.end(), -1);
    for (int64_t i = 0; i < n; ++i) {
        mark[i] = (int32_t)i;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            for (int32_t p = ri[e]; mark[p] != i; p = S.parent[p]) {
                mark[p] = (int32_t)i;
                if (islast[p]) S.rows[cur[S.snode[p]]++] = (int32_t)i;
            }
    }
    S.lptr.assign(ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s) {
        int64_t w = S.super_ptr[s + 1] - S.super_ptr[s], m = S.rptr[s + 1] - S.rptr[s];
        S.lptr[s + 1] = S.lptr[s] + w * m;
        S.max_w = std::max(S.max_w, w);
        S.max_m = std::max(S.max_m, m);
    }

    // ---- levels (height in the supernodal tree) ---------------------------
    S.level.assign(ns, 0);
    S.nlevels = ns ? 1 : 0;
    for (int32_t s = 0; s < ns; ++s) {
        int32_t p = S.sparent[s];
        if (p != -1) S.level[p] = std::max(S.level[p], S.level[s] + 1);
        S.nlevels = std::max(S.nlevels, S.level[s] + 1);
    }

    // ---- assembly map -------------------------------------------------------
    S.amap.resize(S.nnzA);
    S.dsrc.assign(n, 0);
    for (int64_t c = 0; c < n; ++c)
        for (int64_t k = colptr[c]; k < colptr[c + 1]; ++k) {
            int32_t a = S.iperm[rowidx[k]], b = S.iperm[c];
            if (a == b) S.dsrc[a] = k;
            int32_t row = std::max(a, b), col = std::min(a, b);
            int32_t s = S.snode[col];
            int64_t m = S.rptr[s + 1] - S.rptr[s];
            int64_t pos = find_pos(S.rows.data() + S.rptr[s], m, row);
            if (pos < 0) return SPC_INVALID_INPUT;  // cannot happen for a valid pattern
            S.amap[k] = S.lptr[s] + (int64_t)(col - S.super_ptr[s]) * m + pos;
        }

    // ---- full symmetric CSR (caller's ordering) for refinement -------------
    S.csr_ptr.assign(n + 1, 0);
    for (int64_t c = 0; c < n; ++c)
        for (int64_t k = colptr[c]; k < colptr[c + 1]; ++k) {
            S.csr_ptr[rowidx[k] + 1]++;
            if (rowidx[k] != c) S.csr_ptr[c + 1]++;
        }
    for (int64_t i = 0; i < n; ++i) S.csr_ptr[i + 1] += S.csr_ptr[i];
    S.csr_col.resize(S.csr_ptr[n]);
    S.csr_val.resize(S.csr_ptr[n]);
    {
        std::vector<int64_t> fill(S.csr_ptr.begin(), S.csr_ptr.end() - 1);
        for (int64_t c = 0; c < n; ++c)
            for (int64_t k = colptr[c]; k < colptr[c + 1]; ++k) {
                int32_t r = rowidx[k];
                S.csr_col[fill[r]] = (int32_t)c;
                S.csr_val[fill[r]++] = k;
                if (r != c) {
                    S.csr_col[fill[c]] = r;
                    S.csr_val[fill[c]++] = k;
                }
            }
    }

    return build_schedule(S);
}

// Relative indices, scatter pairs, the factor schedule and the solve
// schedule, from the structural arrays of S (super_ptr, snode, sparent,
// parent, rptr, rows, lptr, level, nlevels).
int build_schedule(Symbolic &S) {
    const int64_t n = S.n;
    const int32_t ns = S.nsuper;
    S.pair_ptr.clear();
    S.pairs.clear();
    S.colpair.clear();
    S.rel.clear();
    S.steps.clear();
    S.potrf_tasks.clear();
    S.trsm_tiles.clear();
    S.int_tiles.clear();
    S.ext_tiles.clear();
    S.ext_tiles_big.clear();
    S.trail_big.clear();
    S.ext_flops.clear();
    S.ext_big_flops.clear();
    S.sblocks.clear();
    S.sblock_order.clear();
    S.first_blk.clear();
    S.stasks.clear();
    (void)n;
    // ---- scatter pairs and relative indices -------------------------------
    S.pair_ptr.assign(ns + 1, 0);
    S.colpair.assign(S.rptr[ns], -1);
    for (int32_t s = 0; s < ns; ++s) {
        int64_t w = S.super_ptr[s + 1] - S.super_ptr[s], m = S.rptr[s + 1] - S.rptr[s];
        const int32_t *R = S.rows.data() + S.rptr[s];
        int64_t i = w;
        while (i < m) {
            int32_t t = S.snode[R[i]];
            int64_t i1 = i;
            while (i1 < m && S.snode[R[i1]] == t) ++i1;
            UpdatePair pr;
            pr.target = t;
            pr.i0 = (int32_t)i;
            pr.i1 = (int32_t)i1;
            pr.pad = 0;
            pr.rel_off = (int64_t)S.rel.size();
            const int32_t *Rt = S.rows.data() + S.rptr[t];
            int64_t mt = S.rptr[t + 1] - S.rptr[t], q = 0;
            for (int64_t k = i; k < m; ++k) {  // merge: R_s[i:] is a subset of R_t
                while (q < mt && Rt[q] < R[k]) ++q;
                if (q == mt || Rt[q] != R[k]) return SPC_INVALID_INPUT;  // cannot happen
                S.rel.push_back((int32_t)q);
            }
            for (int64_t k = i; k < i1; ++k) S.colpair[S.rptr[s] + k] = (int32_t)S.pairs.size();
            S.pairs.push_back(pr);
            i = i1;
        }
        S.pair_ptr[s + 1] = (int64_t)S.pairs.size();
    }
    S.cbase.assign(S.rptr[ns], 0);
    S.crel.assign(S.rptr[ns], 0);
    for (int32_t s = 0; s < ns; ++s) {
        int64_t w = S.super_ptr[s + 1] - S.super_ptr[s], m = S.rptr[s + 1] - S.rptr[s];
        for (int64_t k = w; k < m; ++k) {
            const UpdatePair &pr = S.pairs[S.colpair[S.rptr[s] + k]];
            const int32_t t = pr.target;
            S.cbase[S.rptr[s] + k] =
                S.lptr[t] + (int64_t)(S.rows[S.rptr[s] + k] - S.super_ptr[t]) * (S.rptr[t + 1] - S.rptr[t]);
            S.crel[S.rptr[s] + k] = pr.rel_off - pr.i0;
        }
    }

    // ---- column blocks and the inverse store ------------------------------
    std::vector<int32_t> first_blk(ns + 1, 0);
    for (int32_t s = 0; s < ns; ++s) {
        int64_t w = S.super_ptr[s + 1] - S.super_ptr[s];
        first_blk[s] = (int32_t)S.sblocks.size();
        for (int64_t c0 = 0; c0 < w; c0 += kNB)
            S.sblocks.push_back(SolveBlock{s, (int32_t)c0, (int32_t)std::min<int64_t>(c0 + kNB, w), 0});
    }
    first_blk[ns] = (int32_t)S.sblocks.size();
    S.first_blk = first_blk;
    const int64_t nb = (int64_t)S.sblocks.size();
    S.inv_off.assign(nb + 1, 0);
    for (int64_t q = 0; q < nb; ++q) {
        int64_t d = S.sblocks[q].c1 - S.sblocks[q].c0;
        S.inv_off[q + 1] = S.inv_off[q] + d * d;
    }

    // ---- factor schedule ----------------------------------------------------
    // level l: for each block index b, POTRF of block b of every supernode
    // of the level that has it, TRSM tiles of the rows below, trailing SYRK
    // tiles inside the supernode; then the scatter tiles of the level.
    std::vector<std::vector<int32_t>> bylevel(S.nlevels);
    for (int32_t s = 0; s < ns; ++s) bylevel[S.level[s]].push_back(s);
    S.level_step_ptr.assign(S.nlevels + 1, 0);
    S.ext_tile_ptr.assign(S.nlevels + 1, 0);
    S.ext_big_ptr.assign(S.nlevels + 1, 0);
    S.small_ptr.assign(S.nlevels + 1, 0);
    S.small_tasks.clear();
    S.small_flops.assign(S.nlevels, 0.0);
    S.tiny_ptr.assign(S.nlevels + 1, 0);
    S.tiny_tasks.clear();
    S.tiny_flops.assign(S.nlevels, 0.0);
    S.tiny_e16.assign(S.nlevels, 0);
    S.tiny_e32.assign(S.nlevels, 0);
    const Tuning &tu = S.tune;
    auto is_tiny = [&](int32_t s) {
        return S.super_ptr[s + 1] - S.super_ptr[s] <= tu.tiny_w && S.rptr[s + 1] - S.rptr[s] <= tu.tiny_m;
    };
    // lanes per tiny supernode: 16 or 32 (groups sharing a wave), else 64
    auto group_of = [&](int32_t s) {
        const int32_t w = S.super_ptr[s + 1] - S.super_ptr[s];
        const int64_t m = S.rptr[s + 1] - S.rptr[s];
        if (!tu.group || w > kGroupW) return 64;
        return m <= 16 ? 16 : (m <= 32 ? 32 : 64);
    };
    auto is_small = [&](int32_t s) {
        return is_tiny(s) ||
               (S.super_ptr[s + 1] - S.super_ptr[s] <= tu.small_w && S.rptr[s + 1] - S.rptr[s] <= tu.small_m);
    };
    // small subtrees: a supernode that is small and whose children all head
    // small subtrees (children come before their parent in postorder)
    std::vector<char> allsmall(ns, 0);
    for (int32_t s = 0; s < ns; ++s) allsmall[s] = tu.persist && is_small(s);
    for (int32_t s = 0; s < ns; ++s) {
        const int32_t p = S.sparent[s];
        if (p >= 0 && !allsmall[s]) allsmall[p] = 0;
    }
    S.psmall.clear();
    S.ptiny.clear();
    S.pqueue.clear();
    S.persist_flops = 0.0;
    S.pdep0.assign(ns, 0);
    S.ptgt_ptr.assign(ns + 1, 0);
    S.ptgt.clear();
    for (int32_t s = 0; s < ns; ++s) {
        if (allsmall[s])
            for (int64_t q = S.pair_ptr[s]; q < S.pair_ptr[s + 1]; ++q) {
                const int32_t t = S.pairs[q].target;
                if (!allsmall[t]) continue;
                S.ptgt.push_back(t);
                S.pdep0[t]++;
            }
        S.ptgt_ptr[s + 1] = (int64_t)S.ptgt.size();
    }
    S.pchunk.assign(1, 0);
    for (int32_t l = 0; l < S.nlevels; ++l) {
        std::vector<int32_t> big;
        const int32_t level_first = (int32_t)S.pqueue.size();
        // the level's tiny tasks by lanes (16, 32, 64): per-level path (lt)
        // and persistent launch (pt)
        std::vector<SmallTask> lt[3], pt[3];
        auto lanes_slot = [&](int32_t s) {
            const int g = group_of(s);
            return g == 16 ? 0 : (g == 32 ? 1 : 2);
        };
        for (int32_t s : bylevel[l]) {
            if (allsmall[s]) {
                const int32_t wi = S.super_ptr[s + 1] - S.super_ptr[s];
                const int64_t mi = S.rptr[s + 1] - S.rptr[s];
                const SmallTask tk{S.lptr[s], S.rptr[s], S.inv_off[first_blk[s]], s, (int32_t)mi, wi, S.super_ptr[s]};
                const double w = wi, m = (double)mi;
                S.persist_flops += w * w * w / 3.0 + w * w / 2.0 + w / 6.0 + (m - w) * w * w + (m - w) * (m - w + 1) * w;
                if (is_tiny(s)) {
                    pt[lanes_slot(s)].push_back(tk);
                } else {
                    S.pqueue.push_back(PersistEntry{0, (int32_t)S.psmall.size(), 1, 0});
                    S.psmall.push_back(tk);
                }
                continue;
            }
            if (is_small(s)) {
                const int32_t wi = S.super_ptr[s + 1] - S.super_ptr[s];
                const int64_t mi = S.rptr[s + 1] - S.rptr[s];
                const bool tiny = is_tiny(s);
                const SmallTask tk{S.lptr[s], S.rptr[s], S.inv_off[first_blk[s]], s, (int32_t)mi, wi, S.super_ptr[s]};
                if (tiny) {
                    lt[lanes_slot(s)].push_back(tk);
                } else {
                    S.small_tasks.push_back(tk);
                }
                // POTRF + TRSM + SYRK of the rows below (LAPACK counts)
                const double w = wi, m = (double)mi;
                (tiny ? S.tiny_flops : S.small_flops)[l] += w * w * w / 3.0 + w * w / 2.0 + w / 6.0 +
                                                            (m - w) * w * w + (m - w) * (m - w + 1) * w;
            } else {
                big.push_back(s);
            }
        }
        S.small_ptr[l + 1] = (int64_t)S.small_tasks.size();
        S.tiny_tasks.insert(S.tiny_tasks.end(), lt[0].begin(), lt[0].end());
        S.tiny_e16[l] = (int64_t)S.tiny_tasks.size();
        S.tiny_tasks.insert(S.tiny_tasks.end(), lt[1].begin(), lt[1].end());
        S.tiny_e32[l] = (int64_t)S.tiny_tasks.size();
        S.tiny_tasks.insert(S.tiny_tasks.end(), lt[2].begin(), lt[2].end());
        S.tiny_ptr[l + 1] = (int64_t)S.tiny_tasks.size();
        // the level's persistent tiny entries (the supernodes of one level
        // do not depend on each other, so their order inside it is free):
        // kind 2 holds up to 16 in groups of 16 lanes, kind 3 up to 8 in
        // groups of 32, kind 1 up to 4, one wave each
        for (int k = 0; k < 3; ++k) {
            const int32_t kind = k == 0 ? 2 : (k == 1 ? 3 : 1), cap = k == 0 ? 16 : (k == 1 ? 8 : 4);
            for (size_t i = 0; i < pt[k].size(); i += cap) {
                const int32_t cnt = (int32_t)std::min<size_t>(cap, pt[k].size() - i);
                S.pqueue.push_back(PersistEntry{kind, (int32_t)S.ptiny.size(), cnt, 0});
                S.ptiny.insert(S.ptiny.end(), pt[k].begin() + i, pt[k].begin() + i + cnt);
            }
        }
        {
            // chunks of this level's entries: at least about 4096 of them
            // (twice the workgroups the device holds) while chunks hold
            // at most 16 entries
            const int32_t ne = (int32_t)S.pqueue.size() - level_first;
            const int32_t c = std::max(1, std::min(16, ne / 4096));
            for (int32_t e = level_first + c; e < (int32_t)S.pqueue.size(); e += c) S.pchunk.push_back(e);
            if (ne > 0) S.pchunk.push_back((int32_t)S.pqueue.size());
        }
        bylevel[l].swap(big);
    }
    for (int32_t l = 0; l < S.nlevels; ++l) {
        int64_t maxb = 0;
        for (int32_t s : bylevel[l]) {
            int64_t w = S.super_ptr[s + 1] - S.super_ptr[s];
            maxb = std::max(maxb, (w + kNB - 1) / kNB);
        }
        // handover 2: a step takes the hand-over only where few of its
        // tiles wait (they hold their CUs while the block is factored):
        // eight or more supernodes get one, or the waiting tiles are at most
        // 1.5 of the launch's mean share per XCD; otherwise block b+1's
        // column is updated without waits and gets a TRSM launch of its own
        // The bulk update at the end of a group (step b, K = the group's
        // columns) covers the columns beyond block b+1 on 64x64 tiles.  With
        // lookahead (delay >= 2) only the next group's columns get it in
        // step b; the columns beyond the next group are updated in the
        // next group's other steps (its tiles dealt round-robin over steps
        // b+1 .. b+delay-1), beside their column updates and
        // factorizations.  Those columns are next written by the next
        // group's own bulk update (step b+delay), a later launch, and no
        // step in between reads them, so the result is the same.
        std::vector<std::vector<TileTask>> rest_at(maxb);
        std::vector<double> rest_fl(maxb, 0.0);
        {
            const int64_t d = tu.delay;
            const bool spread = tu.lookahead && d >= 2;
            for (int32_t s : bylevel[l]) {
                const int64_t w = S.super_ptr[s + 1] - S.super_ptr[s], m = S.rptr[s + 1] - S.rptr[s];
                for (int64_t b = 0; b * kNB < w; ++b) {
                    const int64_t c1 = std::min<int64_t>(b * kNB + kNB, w), cx = std::min<int64_t>(c1 + kNB, w);
                    if (c1 >= w) continue;
                    const int64_t k0 = (b - b % d) * kNB, kd = c1 - k0;
                    const bool close = b % d == d - 1 || cx >= w;
                    if (!close || (tu.bulk128 && kd >= kTileBig)) continue;
                    const int64_t cn = spread ? std::min<int64_t>(w, c1 + d * kNB) : w;
                    int64_t t = 0;
                    for (int64_t j0 = c1 + kTile; j0 < w; j0 += kTile)
                        for (int64_t i0 = j0; i0 < m; i0 += kTile) {
                            const int64_t at = j0 < cn ? b : b + 1 + (t++ % (d - 1));
                            rest_at[at].push_back(TileTask{S.lptr[s], S.rptr[s], s, (int32_t)m, (int32_t)i0,
                                                           (int32_t)j0, (int32_t)k0, (int32_t)c1, (int32_t)w, -1, -1,
                                                           0});
                            // flops: SYRK on a diagonal tile, GEMM below it
                            const double r = (double)(std::min<int64_t>(i0 + kTile, m) - i0),
                                         c = (double)(std::min<int64_t>(j0 + kTile, w) - j0);
                            rest_fl[at] += i0 == j0 ? (double)kd * (c * (c + 1) + 2.0 * (r - c) * c)
                                                    : 2.0 * (double)kd * r * c;
                        }
                }
            }
        }
        std::vector<char> fuse_step(maxb, 0);
        for (int64_t b = 0; b < maxb; ++b) {
            if (tu.handover == 1) {
                fuse_step[b] = 1;
                continue;
            }
            if (tu.handover != 2) continue;
            int64_t B = 0, nsup = 0;
            for (int32_t s : bylevel[l]) {
                const int64_t w = S.super_ptr[s + 1] - S.super_ptr[s], m = S.rptr[s + 1] - S.rptr[s];
                const int64_t c1 = std::min<int64_t>(b * kNB + kNB, w), cx = std::min<int64_t>(c1 + kNB, w);
                if (b * kNB >= w || c1 >= w) continue;
                ++nsup;
                B += (m - cx + kTile - 1) / kTile;
            }
            const int64_t R = (int64_t)rest_at[b].size();
            fuse_step[b] = nsup >= 8 || 8 * B <= 3 * (R + B) / 2;
        }
        for (int64_t b = 0; b < maxb; ++b) {
            Symbolic::Step st;
            st.potrf_flops = 0.0;
            st.trsm_flops = 0.0;
            st.look_flops = 0.0;
            st.rest_flops = 0.0;
            st.big_flops = 0.0;
            st.q0 = (int64_t)S.trail_big.size();
            st.f0 = (int64_t)S.potrf_tasks.size();
            st.p0 = (int64_t)S.trsm_tiles.size();
            st.t0 = (int64_t)S.int_tiles.size();
            // Blocks go in groups of tu.delay.  Inside a group, step b brings
            // block b+1's columns up to date with the group's panels so far
            // (one column of tiles, K = the group's columns up to b) and
            // factors block b+1 in that column's diagonal tile; the last step
            // of a group updates every column beyond with all of the group's
            // panels at once (K = tu.delay blocks).
            // The trailing launch holds the diagonal tiles of block b+1 first
            // (which also factor it), then the columns beyond block b+1 and
            // the tiles below block b+1's diagonal.  When block b+1 is a full
            // kNB wide, those tiles also do its TRSM, panel by panel as the
            // block is factored, so that block gets no TRSM launch of its
            // own; the block's factorization is claimed by the first of its
            // workgroups to arrive (k_tiles), so no tile ever waits for one
            // that has not started.
            const int64_t gb = b - b % tu.delay;  // first block of b's group
            const bool bulk = b % tu.delay == tu.delay - 1;
            std::vector<TileTask> diag, rest(rest_at[b]), below;
            st.rest_flops += rest_fl[b];
            std::vector<int32_t> below_diag;  // diagonal tile of each waiting tile (index into diag)
            for (int32_t s : bylevel[l]) {
                int64_t w = S.super_ptr[s + 1] - S.super_ptr[s], m = S.rptr[s + 1] - S.rptr[s];
                int64_t c0 = b * kNB;
                if (c0 >= w) continue;
                int64_t c1 = std::min<int64_t>(c0 + kNB, w);
                int32_t blk = first_blk[s] + (int32_t)b;
                const double nbd = (double)(c1 - c0);
                const int64_t cx = std::min<int64_t>(c1 + kNB, w);  // end of block b+1
                const int64_t k0 = gb * kNB;                         // the group's first column
                const double kd = (double)(c1 - k0);
                // the last block of a supernode closes its group too
                const bool close = bulk || cx >= w;
                // block b+1 gets its TRSM from this step's tiles below its
                // diagonal; block b got it from step b-1's
                const bool fuse_next = fuse_step[b] && c1 < w && cx - c1 == kNB;
                const bool fused_here = b > 0 && fuse_step[b - 1] && c1 - c0 == kNB;
                const int32_t gnext = (int32_t)(S.super_ptr[s] + c1);
                // flop counts: POTRF nb^3/3 + nb^2/2 + nb/6, TRSM r nb^2,
                // SYRK k n(n+1), GEMM 2 m n k
                const double nx = (double)(cx - c1), tot = (double)(w - c1);
                if (c1 < w)  // block b+1's POTRF runs in this step's column update
                    st.look_flops += nx * nx * nx / 3.0 + nx * nx / 2.0 + nx / 6.0;
                st.look_flops += nx * (nx + 1) * kd + 2.0 * ((double)(m - c1) - nx) * nx * kd;
                if (fuse_next) st.look_flops += (double)(m - cx) * nx * nx;
                // the bulk update on 128x128 tiles in a launch of its own
                // (K of the group at least 128)
                const bool to128 = tu.bulk128 && c1 - k0 >= kTileBig;
                if (close && to128)
                    st.big_flops += tot * (tot + 1) * kd + 2.0 * (double)(m - w) * tot * kd -
                                    (nx * (nx + 1) * kd + 2.0 * ((double)(m - c1) - nx) * nx * kd);
                // block 0 gets a POTRF task; block b+1 is factored by the
                // workgroup of its diagonal tile in step b's column update
                if (b == 0) {
                    st.potrf_flops += nbd * nbd * nbd / 3.0 + nbd * nbd / 2.0 + nbd / 6.0;
                    S.potrf_tasks.push_back(PanelTask{S.lptr[s], S.inv_off[blk], s, (int32_t)m, (int32_t)c0,
                                                      (int32_t)c1, (int32_t)(S.super_ptr[s] + c0), 0});
                }
                if (!fused_here) {
                    st.trsm_flops += (double)(m - c1) * nbd * nbd;
                    for (int64_t r = c1; r < m; r += kTile)
                        S.trsm_tiles.push_back(TileTask{S.lptr[s], S.inv_off[blk], s, (int32_t)m, (int32_t)r,
                                                        (int32_t)c0, (int32_t)c0, (int32_t)c1, (int32_t)c1, blk, -1,
                                                        0});
                }
                if (c1 >= w) continue;
                const int32_t di = (int32_t)diag.size();
                diag.push_back(TileTask{S.lptr[s], S.inv_off[blk + 1], s, (int32_t)m, (int32_t)c1, (int32_t)c1,
                                        (int32_t)k0, (int32_t)c1, (int32_t)w, gnext, fuse_next ? blk + 1 : -1, 0});
                if (close && to128)
                    for (int64_t j0 = c1 + kTile; j0 < w; j0 += kTileBig)
                        for (int64_t i0 = j0; i0 < m; i0 += kTileBig)
                            S.trail_big.push_back(TileTask{S.lptr[s], S.rptr[s], s, (int32_t)m, (int32_t)i0,
                                                           (int32_t)j0, (int32_t)k0, (int32_t)c1, (int32_t)w, -1,
                                                           -1, 0});
                // (the columns beyond block b+1 otherwise: rest_at)
                // block b+1's columns below its diagonal tile
                for (int64_t i0 = c1 + kTile; i0 < m; i0 += kTile) {
                    const TileTask tt{S.lptr[s], fuse_next ? S.inv_off[blk + 1] : S.rptr[s], s, (int32_t)m,
                                      (int32_t)i0, (int32_t)c1, (int32_t)k0, (int32_t)c1, (int32_t)w,
                                      fuse_next ? gnext : -1, fuse_next ? blk + 1 : -1, 0};
                    if (fuse_next) {
                        below.push_back(tt);
                        below_diag.push_back(di);
                    } else {
                        rest.push_back(tt);
                    }
                }
            }
            // layout: the diagonal tiles, then per residue r of the launch
            // index (mod 8, one XCD) a queue of other tiles followed by the
            // waiting tiles whose diagonal tile has residue r, emitted by
            // position; the other tiles are spread so that every residue
            // holds about as many tiles (water-filling), since the waiting
            // tiles of a supernode all land on one XCD.  Safety does not rest
            // on this placement (a wait is only ever on a running workgroup:
            // k_tiles); it keeps the hand-over within one XCD's L2, which
            // measured faster (60^3: 12.3 ms against 12.9 with the waiting
            // tiles spread over the XCDs after the other tiles)
            const int64_t nd = (int64_t)diag.size();
            std::vector<std::vector<const TileTask *>> qr(8);
            {
                int64_t c[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                for (int32_t di : below_diag) c[(di % 8)]++;
                // residues start after the diagonal tiles: position nd is residue nd % 8
                const int64_t R = (int64_t)rest.size();
                int64_t lo = 0, hi = R + (int64_t)below.size() + 1;  // smallest T with sum max(0, T - c) >= R
                while (lo < hi) {
                    const int64_t T = (lo + hi) / 2;
                    int64_t sum = 0;
                    for (int r = 0; r < 8; ++r) sum += std::max<int64_t>(0, T - c[r]);
                    if (sum >= R) hi = T;
                    else lo = T + 1;
                }
                int64_t take[8], left = R;
                for (int r = 0; r < 8; ++r) take[r] = std::max<int64_t>(0, lo - 1 - c[r]);
                for (int r = 0; r < 8; ++r) left -= take[r];
                for (int r = 0; r < 8 && left > 0; ++r)
                    if (lo - c[r] > take[r] && lo - c[r] > 0) {
                        ++take[r];
                        --left;
                    }
                size_t ri = 0;
                for (int r = 0; r < 8; ++r)
                    for (int64_t e = 0; e < take[r]; ++e) qr[r].push_back(&rest[ri++]);
                for (; ri < rest.size(); ++ri) qr[ri % 8].push_back(&rest[ri]);  // (never: the takes add to R)
                for (size_t e = 0; e < below.size(); ++e) qr[below_diag[e] % 8].push_back(&below[e]);
            }
            for (const TileTask &tt : diag) S.int_tiles.push_back(tt);
            st.tm = (int64_t)S.int_tiles.size();
            {
                const TileTask noop{0, 0, -1, 1, 0, 0, 0, 0, 0, -1, -1, 0};
                std::vector<size_t> qi(8, 0);
                size_t pending = 0;
                for (auto &q : qr) pending += q.size();
                for (int64_t pos = nd; pending > 0; ++pos) {
                    const int r = (int)(pos % 8);
                    if (qi[r] < qr[r].size()) {
                        S.int_tiles.push_back(*qr[r][qi[r]++]);
                        --pending;
                    } else {
                        S.int_tiles.push_back(noop);
                    }
                }
            }
            st.f1 = (int64_t)S.potrf_tasks.size();
            st.p1 = (int64_t)S.trsm_tiles.size();
            st.t1 = (int64_t)S.int_tiles.size();
            st.q1 = (int64_t)S.trail_big.size();
            S.steps.push_back(st);
        }
        S.level_step_ptr[l + 1] = (int64_t)S.steps.size();
        double ef = 0.0, efb = 0.0;
        for (int32_t s : bylevel[l]) {
            int64_t w = S.super_ptr[s + 1] - S.super_ptr[s], m = S.rptr[s + 1] - S.rptr[s];
            const bool big = m - w >= tu.big_min && w >= tu.big_min_k;
            (big ? efb : ef) += (double)(m - w) * (double)(m - w + 1) * (double)w;
            const int64_t tsz = big ? kTileBig : kTile;
            for (int64_t j0 = w; j0 < m; j0 += tsz)
                for (int64_t i0 = j0; i0 < m; i0 += tsz)
                    (big ? S.ext_tiles_big : S.ext_tiles)
                        .push_back(TileTask{S.lptr[s], S.rptr[s], s, (int32_t)m, (int32_t)i0, (int32_t)j0, 0,
                                            (int32_t)w, (int32_t)m, -1, -1, 0});
        }
        S.ext_tile_ptr[l + 1] = (int64_t)S.ext_tiles.size();
        S.ext_big_ptr[l + 1] = (int64_t)S.ext_tiles_big.size();
        S.ext_flops.push_back(ef);
        S.ext_big_flops.push_back(efb);
    }

    // ---- solve schedule: block-tree levels ---------------------------------
    // parent of block q: the next block of its supernode, else the block of
    // the parent supernode holding the parent column of the last column
    std::vector<int32_t> blev(nb, 0);
    int32_t nsl = nb ? 1 : 0;
    for (int64_t q = 0; q < nb; ++q) {
        const SolveBlock &B = S.sblocks[q];
        int64_t w = S.super_ptr[B.s + 1] - S.super_ptr[B.s];
        int64_t pq = -1;
        if (B.c1 < w) pq = q + 1;
        else {
            int32_t pc = S.parent[S.super_ptr[B.s + 1] - 1];
            if (pc != -1) {
                int32_t t = S.snode[pc];
                pq = first_blk[t] + (pc - S.super_ptr[t]) / kNB;
            }
        }
        if (pq != -1) blev[pq] = std::max(blev[pq], blev[q] + 1);
        nsl = std::max(nsl, blev[q] + 1);
    }
    S.nslevels = nsl;
    S.slevel_ptr.assign(nsl + 1, 0);
    for (int64_t q = 0; q < nb; ++q) S.slevel_ptr[blev[q] + 1]++;
    for (int32_t l = 0; l < nsl; ++l) S.slevel_ptr[l + 1] += S.slevel_ptr[l];
    S.sblock_order.resize(nb);
    {
        std::vector<int64_t> f(S.slevel_ptr.begin(), S.slevel_ptr.end() - 1);
        for (int64_t q = 0; q < nb; ++q) S.sblock_order[f[blev[q]]++] = (int32_t)q;
    }
    // one task per chunk of rows below the block; a block with no rows
    // below still gets one (empty) task, which does its diagonal part.
    // Levels from the top with fewer than solve_persist_max tasks run
    // persistently (solve_split..); below them, the blocks of tiny
    // supernodes (a single block and a single task) go to the one-wave
    // solve kernels instead.
    auto block_tasks = [&](const SolveBlock &B) {
        const int64_t m = S.rptr[B.s + 1] - S.rptr[B.s];
        return std::max<int64_t>(1, (m - B.c1 + kSolveRows - 1) / kSolveRows);
    };
    int32_t split = nsl;
    for (; split > 0; --split) {
        int64_t cnt = 0;
        for (int64_t e = S.slevel_ptr[split - 1]; e < S.slevel_ptr[split]; ++e)
            cnt += block_tasks(S.sblocks[S.sblock_order[e]]);
        if (cnt >= tu.solve_persist_max) break;
    }
    S.solve_split = split;
    S.stask_ptr.assign(nsl + 1, 0);
    S.stiny_ptr.assign(nsl + 1, 0);
    S.stiny.clear();
    for (int32_t l = 0; l < nsl; ++l) {
        for (int64_t e = S.slevel_ptr[l]; e < S.slevel_ptr[l + 1]; ++e) {
            int32_t q = S.sblock_order[e];
            SolveBlock &B = S.sblocks[q];
            int64_t m = S.rptr[B.s + 1] - S.rptr[B.s];
            const int64_t w = S.super_ptr[B.s + 1] - S.super_ptr[B.s];
            if (l < split && w <= tu.tiny_w && m <= tu.tiny_m) {
                S.stiny.push_back(SmallTask{S.lptr[B.s], S.rptr[B.s], S.inv_off[q], B.s, (int32_t)m, (int32_t)w,
                                            S.super_ptr[B.s]});
                B.ntasks = 1;
                continue;
            }
            const size_t first = S.stasks.size();
            int32_t cnt = 0;
            int64_t r = B.c1;
            do {
                int64_t r1 = std::min<int64_t>(r + kSolveRows, m);
                SolveTask tk;
                tk.loff = S.lptr[B.s];
                tk.roff = S.rptr[B.s];
                tk.ioff = S.inv_off[q];
                tk.g0 = S.super_ptr[B.s] + B.c0;
                tk.m = (int32_t)m;
                tk.c0 = B.c0;
                tk.nb = B.c1 - B.c0;
                tk.r0 = (int32_t)r;
                tk.r1 = (int32_t)r1;
                tk.blk = q;
                tk.first = cnt == 0;
                tk.hand = 0;
                tk.pad = 0;
                S.stasks.push_back(tk);
                ++cnt;
                r = r1;
            } while (r < m);
            B.ntasks = cnt;
            for (size_t e = first; e < S.stasks.size(); ++e) S.stasks[e].ntasks = cnt;
        }
        S.stask_ptr[l + 1] = (int64_t)S.stasks.size();
        S.stiny_ptr[l + 1] = (int64_t)S.stiny.size();
    }
    // dependencies of the persistent solves
    {
        std::vector<int32_t> col_blk(S.n);
        for (int32_t s = 0; s < ns; ++s)
            for (int32_t c = S.super_ptr[s]; c < S.super_ptr[s + 1]; ++c)
                col_blk[c] = first_blk[s] + (c - S.super_ptr[s]) / kNB;
        const int64_t nt = (int64_t)S.stasks.size();
        const int64_t tp0 = S.stask_ptr[split];
        S.stgt_ptr.assign(nt + 1, 0);
        S.stgt.clear();
        S.fdep.assign(nb, 0);
        for (int64_t t = 0; t < nt; ++t) {
            const SolveTask &tk = S.stasks[t];
            int32_t last = -1;
            for (int64_t r = tk.r0; r < tk.r1; ++r) {
                const int32_t b = col_blk[S.rows[tk.roff + r]];
                if (b != last) {
                    S.stgt.push_back(b);
                    if (t >= tp0) S.fdep[b]++;
                    last = b;
                }
            }
            S.stgt_ptr[t + 1] = (int64_t)S.stgt.size();
        }
        // hand-over inside a supernode: the first task of block q - 1 covers
        // q's rows first (its rows start right below q - 1), so in the
        // persistent sweeps it passes q's sums (forward) and takes x_q
        // (backward) through buffers polled for a value, which spares the
        // counter or flag round trip on the chain from block to block
        {
            std::vector<int64_t> first_of(nb, -1);
            for (int64_t t = tp0; t < nt; ++t)
                if (S.stasks[t].first) first_of[S.stasks[t].blk] = t;
            for (int64_t q = 1; q < nb; ++q) {
                const SolveBlock &B = S.sblocks[q];
                if (B.c0 == 0 || first_of[q] < 0 || first_of[q - 1] < 0) continue;
                SolveTask &prev = S.stasks[first_of[q - 1]];
                prev.hand |= kHandOut | ((B.c1 - B.c0) << 8);
                for (int64_t t = first_of[q]; t < first_of[q] + S.stasks[first_of[q]].ntasks; ++t)
                    S.stasks[t].hand |= kHandIn;
                S.fdep[q]--;
            }
        }
        // backward order: levels from the top; inside a level, each block's
        // other tasks and then its first task, which finishes the block (it
        // holds the rows nearest the block, whose x come last)
        S.bwd_order.clear();
        for (int32_t l = nsl - 1; l >= split; --l)
            for (int64_t e = S.stask_ptr[l]; e < S.stask_ptr[l + 1]; e += S.stasks[e].ntasks) {
                for (int32_t k = 1; k < S.stasks[e].ntasks; ++k) S.bwd_order.push_back((int32_t)(e + k));
                S.bwd_order.push_back((int32_t)e);
            }
    }
    return SPC_OK;
}

// Disjoint union of analyses: system i's columns, supernodes, rows and
// panel entries follow those of systems 0..i-1; its caller entries follow
// theirs too.  The schedule is then built for the whole forest, so level l
// of the union holds level l of every system.
int verify_schedule(const Symbolic &S, std::string &msg) {
    auto fail = [&](const char *what, int64_t a, int64_t b) {
        char buf[200];
        std::snprintf(buf, sizeof(buf), "%s (%lld, %lld)", what, (long long)a, (long long)b);
        msg = buf;
        return -1;
    };
    const int64_t nb = (int64_t)S.sblocks.size();
    // rows below each block solved by a TRSM launch or by hand-over tiles
    std::vector<int64_t> solved(nb, 0);
    std::vector<char> blocked(S.nsuper, 0);
    for (const PanelTask &pt : S.potrf_tasks) blocked[pt.s] = 1;
    auto block_of = [&](int32_t s, int64_t c) { return (int64_t)S.first_blk[s] + c / kNB; };
    auto m_of = [&](int32_t s) { return S.rptr[s + 1] - S.rptr[s]; };
    for (const TileTask &tt : S.trsm_tiles) {
        if (tt.s < 0 || tt.s >= S.nsuper || tt.blk < 0 || tt.blk >= nb) return fail("TRSM tile out of range", tt.s, tt.blk);
        solved[tt.blk] += std::min<int64_t>(tt.i0 + kTile, m_of(tt.s)) - tt.i0;
    }
    std::vector<int64_t> dpos(nb, -1);
    for (const Symbolic::Step &st : S.steps) {
        for (int64_t t = st.t0; t < st.t1; ++t) {
            const TileTask &tt = S.int_tiles[t];
            if (tt.s < 0) {  // no-op entry
                if (tt.flag != -1 || t < st.tm) return fail("no-op entry misplaced", t, tt.flag);
                continue;
            }
            if (tt.s >= S.nsuper || tt.loff != S.lptr[tt.s] || tt.m != m_of(tt.s))
                return fail("trailing tile of an unknown supernode", t, tt.s);
            const bool diag = tt.blk >= 0 && tt.i0 == tt.j0;
            if (diag) {
                if (t >= st.tm) return fail("diagonal tile after the others", t, st.tm);
                if (tt.flag >= 0) {
                    const int64_t q = block_of(tt.s, tt.j0);
                    if (tt.flag != q || S.sblocks[q].c1 - S.sblocks[q].c0 != kNB)
                        return fail("hand-over from a block that is not full", t, tt.flag);
                    dpos[q] = t;
                }
            } else if (tt.flag >= 0) {
                const int64_t q = tt.flag;
                if (q >= nb || dpos[q] < st.t0 || dpos[q] >= t) return fail("waiting tile before its diagonal tile", t, q);
                const TileTask &d = S.int_tiles[dpos[q]];
                if (d.s != tt.s || d.j0 != tt.j0 || tt.i0 < tt.j0 + kTile) return fail("waiting tile of another block", t, q);
                // a waiting tile that claims the block's factorization runs
                // the diagonal tile's task rebuilt from its own (i0 = j0)
                if (d.loff != tt.loff || d.aux != tt.aux || d.m != tt.m || d.k0 != tt.k0 || d.k1 != tt.k1 ||
                    d.jmax != tt.jmax || d.blk != tt.blk)
                    return fail("waiting tile whose task does not rebuild its diagonal tile's", t, q);
                solved[q] += std::min<int64_t>(tt.i0 + kTile, tt.m) - tt.i0;
            }
        }
    }
    for (int64_t q = 0; q < nb; ++q) {
        const SolveBlock &b = S.sblocks[q];
        if (!blocked[b.s]) continue;
        if (solved[q] != m_of(b.s) - b.c1) return fail("rows below a block not solved exactly once", q, solved[q]);
    }
    // every supernode is factored by exactly one path
    std::vector<int32_t> seen(S.nsuper, 0);
    for (const SmallTask &t : S.small_tasks) seen[t.s]++;
    for (const SmallTask &t : S.tiny_tasks) seen[t.s]++;
    for (const SmallTask &t : S.psmall) seen[t.s]++;
    for (const SmallTask &t : S.ptiny) seen[t.s]++;
    for (int32_t t = 0; t < S.nsuper; ++t)
        if (seen[t] + (blocked[t] ? 1 : 0) != 1) return fail("supernode not factored exactly once", t, seen[t]);
    // the per-level tiny lists: groups of 16 lanes, then of 32, then one
    // wave each, every supernode within its part's limits
    for (int32_t l = 0; l < S.nlevels; ++l) {
        const int64_t a = S.tiny_ptr[l], b = S.tiny_e16[l], c = S.tiny_e32[l], d = S.tiny_ptr[l + 1];
        if (!(a <= b && b <= c && c <= d)) return fail("tiny lists out of order", l, b);
        for (int64_t q = a; q < c; ++q) {
            const SmallTask &t = S.tiny_tasks[q];
            if (t.w > kGroupW || t.m > (q < b ? 16 : 32)) return fail("supernode does not fit its lane group", t.s, t.m);
        }
        for (int64_t q = a; q < d; ++q)
            if (S.tiny_tasks[q].w > kTinyW || S.tiny_tasks[q].m > kTinyM)
                return fail("supernode beyond the one-wave limits", S.tiny_tasks[q].s, S.tiny_tasks[q].m);
    }
    // persistent launch: every count-down target comes in a later queue
    // entry than its source, and each counter starts at the number of its
    // sources, so a wait only ever waits on entries taken before it
    std::vector<int64_t> pos(S.nsuper, -1);
    for (int64_t e = 0; e < (int64_t)S.pqueue.size(); ++e) {
        const PersistEntry &pe = S.pqueue[e];
        const std::vector<SmallTask> &src = pe.kind == 0 ? S.psmall : S.ptiny;
        const int32_t cap = pe.kind == 0 ? 1 : (pe.kind == 1 ? 4 : (pe.kind == 2 ? 16 : 8));
        if (pe.kind < 0 || pe.kind > 3 || pe.count < 1 || pe.count > cap || pe.first < 0 ||
            pe.first + pe.count > (int32_t)src.size())
            return fail("bad persistent queue entry", e, pe.count);
        for (int32_t k = 0; k < pe.count; ++k) {
            const SmallTask &t = src[pe.first + k];
            // a group entry's supernodes fit their groups
            if (pe.kind >= 2 && (t.w > kGroupW || t.m > (pe.kind == 2 ? 16 : 32)))
                return fail("supernode does not fit its lane group", t.s, t.m);
            pos[t.s] = e;
        }
    }
    if (S.pchunk.empty() || S.pchunk.front() != 0 || S.pchunk.back() != (int32_t)S.pqueue.size())
        return fail("persistent chunks do not cover the queue", (int64_t)S.pchunk.size(), (int64_t)S.pqueue.size());
    for (size_t c = 0; c + 1 < S.pchunk.size(); ++c)
        if (S.pchunk[c + 1] <= S.pchunk[c]) return fail("empty persistent chunk", (int64_t)c, S.pchunk[c]);
    std::vector<int32_t> count(S.nsuper, 0);
    for (int32_t t = 0; t < S.nsuper; ++t) {
        if (pos[t] < 0) {
            if (S.ptgt_ptr[t + 1] != S.ptgt_ptr[t]) return fail("count-down from outside the persistent set", t, 0);
            continue;
        }
        for (int64_t q = S.ptgt_ptr[t]; q < S.ptgt_ptr[t + 1]; ++q) {
            const int32_t u = S.ptgt[q];
            if (pos[u] <= pos[t]) return fail("persistent count-down target not after its source", t, u);
            count[u]++;
        }
    }
    for (int32_t t = 0; t < S.nsuper; ++t)
        if (pos[t] >= 0 && count[t] != S.pdep0[t]) return fail("persistent counter start", t, S.pdep0[t]);
    // persistent solves: a hand-over goes from the first task of block q - 1
    // to every task of block q of the same supernode, over exactly q's rows,
    // which come first in that task; each forward counter starts at the
    // (task, block) contributions of the persistent tasks that do not come
    // through a hand-over
    {
        const int64_t nt = (int64_t)S.stasks.size(), tp0 = S.stask_ptr[S.solve_split];
        std::vector<int32_t> want(nb, 0);
        for (int64_t t = 0; t < nt; ++t) {
            const SolveTask &k = S.stasks[t];
            if (t < tp0) {
                if (k.hand) return fail("hand-over outside the persistent sweeps", t, k.hand);
                continue;
            }
            const bool out = (k.hand & kHandOut) != 0;
            if (out) {
                const int64_t q = k.blk + 1;
                if (!k.first || q >= nb || S.sblocks[q].s != S.sblocks[k.blk].s || k.r0 != S.sblocks[q].c0 ||
                    (k.hand >> 8) != S.sblocks[q].c1 - S.sblocks[q].c0)
                    return fail("hand-over not over the next block's rows", t, k.hand);
            }
            if ((k.hand & kHandIn) != 0) {
                const SolveBlock &B = S.sblocks[k.blk];
                if (B.c0 == 0) return fail("hand-over into a supernode's first block", t, k.blk);
            }
            for (int64_t e = S.stgt_ptr[t]; e < S.stgt_ptr[t + 1]; ++e)
                if (!(out && S.stgt[e] == k.blk + 1)) want[S.stgt[e]]++;
        }
        std::vector<char> hands_out(nb, 0);
        for (int64_t t = tp0; t < nt; ++t)
            if (S.stasks[t].first && (S.stasks[t].hand & kHandOut)) hands_out[S.stasks[t].blk] = 1;
        for (int64_t t = tp0; t < nt; ++t) {
            const SolveTask &k = S.stasks[t];
            const bool in = (k.hand & kHandIn) != 0;
            if (in != (k.blk > 0 && S.sblocks[k.blk].c0 > 0 && hands_out[k.blk - 1]))
                return fail("hand-over flags of two blocks disagree", t, k.blk);
        }
        for (int64_t q = 0; q < nb; ++q)
            if (want[q] != S.fdep[q]) return fail("forward counter start", q, S.fdep[q]);
    }
    return 0;
}

int merge(const std::vector<const Symbolic *> &parts, Symbolic &M, std::vector<int64_t> &col_off,
          std::vector<int64_t> &panel_off, std::vector<int64_t> &inv_base, std::vector<int64_t> &val_off) {
    M = Symbolic();
    const size_t k = parts.size();
    if (k) M.tune = parts[0]->tune;
    col_off.assign(k + 1, 0);
    panel_off.assign(k + 1, 0);
    inv_base.assign(k + 1, 0);
    val_off.assign(k + 1, 0);
    int64_t sn_off = 0, row_off = 0;
    M.super_ptr.push_back(0);
    M.rptr.push_back(0);
    M.lptr.push_back(0);
    M.csr_ptr.push_back(0);
    for (size_t i = 0; i < k; ++i) {
        const Symbolic &S = *parts[i];
        const int64_t c0 = col_off[i], p0 = panel_off[i];
        for (int64_t j = 0; j < S.n; ++j) {
            M.perm.push_back((int32_t)(c0 + S.perm[j]));
            M.iperm.push_back((int32_t)(c0 + S.iperm[j]));
            M.parent.push_back(S.parent[j] < 0 ? -1 : (int32_t)(c0 + S.parent[j]));
            M.colcount.push_back(S.colcount[j]);
            M.snode.push_back((int32_t)(sn_off + S.snode[j]));
        }
        for (int32_t s = 0; s < S.nsuper; ++s) {
            M.super_ptr.push_back((int32_t)(c0 + S.super_ptr[s + 1]));
            M.sparent.push_back(S.sparent[s] < 0 ? -1 : (int32_t)(sn_off + S.sparent[s]));
            M.level.push_back(S.level[s]);
            M.rptr.push_back(row_off + S.rptr[s + 1]);
            M.lptr.push_back(p0 + S.lptr[s + 1]);
        }
        for (int32_t r : S.rows) M.rows.push_back((int32_t)(c0 + r));
        for (int32_t s = 0; s < S.nsuper; ++s) M.status_slot.push_back((int32_t)i);
        for (int64_t a : S.amap) M.amap.push_back(p0 + a);
        for (int64_t d : S.dsrc) M.dsrc.push_back(val_off[i] + d);
        // the full-A CSR of the union: rows and columns shifted by the
        // part's first column, entries by its first caller value
        const int64_t e0 = M.csr_ptr.back();
        for (int64_t r = 0; r < S.n; ++r) M.csr_ptr.push_back(e0 + S.csr_ptr[r + 1]);
        for (int32_t c : S.csr_col) M.csr_col.push_back((int32_t)(c0 + c));
        for (int64_t v : S.csr_val) M.csr_val.push_back(val_off[i] + v);
        M.nnzA += S.nnzA;
        M.flops += S.flops;
        M.nnzL += S.nnzL;
        M.max_w = std::max(M.max_w, S.max_w);
        M.max_m = std::max(M.max_m, S.max_m);
        M.nlevels = std::max(M.nlevels, S.nlevels);
        sn_off += S.nsuper;
        row_off += S.rows_total();
        col_off[i + 1] = c0 + S.n;
        panel_off[i + 1] = p0 + S.panel_entries();
        inv_base[i + 1] = inv_base[i] + (S.inv_off.empty() ? 0 : S.inv_off.back());
        val_off[i + 1] = val_off[i] + S.nnzA;
    }
    M.n = col_off[k];
    M.nsuper = (int32_t)sn_off;
    if (M.n > INT32_MAX - 1) return SPC_INVALID_INPUT;
    return build_schedule(M);
}

}  // namespace spc
