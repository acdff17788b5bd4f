/*
 * oracle.c -- plain FP64 CPU oracle for supernodal sparse Cholesky.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP library.
 *
 * What it computes, and where each step comes from:
 *   - analyze (paper Sec. 2, "Background on CHOLMOD"): symmetric permutation
 *     by a given fill-reducing order, elimination tree, column counts and the
 *     pattern of L, node amalgamation into supernodes.  The pattern is found
 *     by the column-merge recurrence (George & Liu, "Computer Solution of
 *     Large Sparse Positive Definite Systems", 1981):
 *         S_j = { i > j : A_ij != 0 }  U  union over children c of j of (S_c \ {j})
 *         parent(j) = min S_j   (none if S_j is empty)
 *     which is a different algorithm from the library's.
 *   - factorize (Sec. 3, "Task-Based Parallel CHOLMOD", and its Listing 1):
 *     left-looking supernodal loop over supernodes in ascending order; each
 *     supernode is built from A, receives the SYRK/GEMM update of every
 *     earlier supernode that touches its columns, then is factored by a
 *     column Cholesky of the diagonal block and the triangular solve of the
 *     rows below (POTRF + TRSM).  orc_factor_parallel runs the same steps
 *     with whole supernodes per host thread, level by level of the
 *     elimination tree (the one-task-per-supernode scheme of Sec. 3-4), with
 *     a bit-identical result.
 *   - solve (Sec. 1 and Sec. 2): L y = b then L^T x = y, supernode by
 *     supernode, with the permutation applied at entry and exit.
 *
 * Readings where the paper is silent (ordering rule, postorder tie-break,
 * amalgamation rule, pivot-failure rule) are fixed in the function comments.
 * All floating point is double; every sum runs in ascending index order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#define omp_get_num_threads_or_one() omp_get_num_threads()
#else
#define omp_get_num_threads_or_one() 1
#endif

typedef struct orc_sym {
    int64_t n;
    int32_t *perm;       /* final order: perm[k] = original index of pivot k */
    int32_t *iperm;      /* inverse of perm */
    int32_t *post;       /* postorder applied on top of the given order */
    int32_t *parent;     /* elimination tree of the final permuted matrix */
    int32_t *colcount;   /* |struct(L_:j)| including the diagonal */
    int64_t *Lp;         /* exact pattern of L, below the diagonal */
    int32_t *Li;
    /* permuted lower matrix Ahat (CSC, rows sorted) and for each of its
     * entries the position of the source entry in the caller's CSC */
    int64_t *Ap;
    int32_t *Ai;
    int64_t *Amap;
    /* fundamental supernodes */
    int32_t nfund;
    int32_t *fund_ptr;
    /* final (amalgamated) supernodes */
    int32_t nsuper;
    int32_t *super_ptr;  /* [nsuper+1] first column of each supernode */
    int32_t *snode;      /* [n] supernode of each column */
    int32_t *sparent;    /* supernodal parent, -1 for a root */
    int64_t *rptr;       /* [nsuper+1] row lists R_s */
    int32_t *rows;
    int64_t *lptr;       /* [nsuper+1] panel offsets, m_s*w_s each */
    int64_t *uptr;       /* [nsuper+1] update lists U_s (ascending d < s) */
    int32_t *ulist;
    int32_t *level;      /* 0 for leaves, 1 + max over children otherwise */
    int32_t nlevels;
    int64_t flops;       /* sum of colcount^2 */
    int64_t nnzL;        /* sum of colcount */
    int64_t zeros;       /* explicit zeros stored because of amalgamation */
} orc_sym;

static void *xmalloc(size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p) abort();
    return p;
}
static void *xcalloc(size_t count, size_t size) {
    void *p = calloc(count ? count : 1, size ? size : 1);
    if (!p) abort();
    return p;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Ahat = A(perm, perm), lower part, sorted rows; amap[k] = source entry. */
static void permute_lower(int64_t n, const int64_t *colptr, const int32_t *rowidx,
                          const int32_t *iperm, int64_t **Ap_out, int32_t **Ai_out,
                          int64_t **map_out) {
    int64_t nnz = colptr[n];
    int64_t *cnt = xcalloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t c = 0; c < n; ++c)
        for (int64_t k = colptr[c]; k < colptr[c + 1]; ++k) {
            int32_t i = iperm[rowidx[k]], j = iperm[c];
            int32_t col = i < j ? i : j;
            cnt[col + 1]++;
        }
    for (int64_t j = 0; j < n; ++j) cnt[j + 1] += cnt[j];
    int64_t *Ap = xmalloc(sizeof(int64_t) * (n + 1));
    memcpy(Ap, cnt, sizeof(int64_t) * (n + 1));
    int32_t *Ai = xmalloc(sizeof(int32_t) * (size_t)nnz);
    int64_t *map = xmalloc(sizeof(int64_t) * (size_t)nnz);
    int64_t *next = cnt; /* reuse as insertion cursor */
    for (int64_t c = 0; c < n; ++c)
        for (int64_t k = colptr[c]; k < colptr[c + 1]; ++k) {
            int32_t i = iperm[rowidx[k]], j = iperm[c];
            int32_t col = i < j ? i : j, row = i < j ? j : i;
            int64_t dst = next[col]++;
            Ai[dst] = row;
            map[dst] = k;
        }
    /* insertion sort of each column by row (columns are short) */
    for (int64_t j = 0; j < n; ++j)
        for (int64_t a = Ap[j] + 1; a < Ap[j + 1]; ++a) {
            int32_t r = Ai[a];
            int64_t m = map[a], b = a - 1;
            while (b >= Ap[j] && Ai[b] > r) {
                Ai[b + 1] = Ai[b];
                map[b + 1] = map[b];
                --b;
            }
            Ai[b + 1] = r;
            map[b + 1] = m;
        }
    free(cnt);
    *Ap_out = Ap;
    *Ai_out = Ai;
    *map_out = map;
}

/* Column-merge symbolic factorization of the lower matrix (Ap, Ai):
 * fills parent[n] and the strictly-lower pattern (Lp, Li, rows sorted). */
static void column_merge(int64_t n, const int64_t *Ap, const int32_t *Ai, int32_t *parent,
                         int64_t **Lp_out, int32_t **Li_out) {
    int32_t *mark = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *child_head = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *child_next = xmalloc(sizeof(int32_t) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) {
        mark[j] = -1;
        child_head[j] = -1;
    }
    int64_t cap = 4 * n + 16, len = 0;
    int32_t *Li = xmalloc(sizeof(int32_t) * (size_t)cap);
    int64_t *Lp = xmalloc(sizeof(int64_t) * (size_t)(n + 1));
    for (int64_t j = 0; j < n; ++j) {
        Lp[j] = len;
        mark[j] = (int32_t)j;
        /* entries of A strictly below the diagonal */
        for (int64_t k = Ap[j]; k < Ap[j + 1]; ++k) {
            int32_t i = Ai[k];
            if (mark[i] != j) {
                mark[i] = (int32_t)j;
                if (len == cap) { cap *= 2; Li = realloc(Li, sizeof(int32_t) * (size_t)cap); if (!Li) abort(); }
                Li[len++] = i;
            }
        }
        /* structures of the children, without j itself */
        for (int32_t c = child_head[j]; c != -1; c = child_next[c])
            for (int64_t k = Lp[c]; k < Lp[c + 1]; ++k) {
                int32_t i = Li[k];
                if (mark[i] != j) {
                    mark[i] = (int32_t)j;
                    if (len == cap) { cap *= 2; Li = realloc(Li, sizeof(int32_t) * (size_t)cap); if (!Li) abort(); }
                    Li[len++] = i;
                }
            }
        qsort(Li + Lp[j], (size_t)(len - Lp[j]), sizeof(int32_t), cmp_i32);
        parent[j] = (len > Lp[j]) ? Li[Lp[j]] : -1;
        if (parent[j] != -1) {
            /* the union does not depend on the order of the children */
            child_next[j] = child_head[parent[j]];
            child_head[parent[j]] = (int32_t)j;
        }
        Lp[j + 1] = len;
    }
    free(mark);
    free(child_head);
    free(child_next);
    *Lp_out = Lp;
    *Li_out = Li;
}

/* Postorder of a forest: roots ascending, children ascending, numbered in
 * post-visit order.  post[k] = node visited k-th. */
static void postorder(int64_t n, const int32_t *parent, int32_t *post) {
    int32_t *head = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *next = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *stack = xmalloc(sizeof(int32_t) * (size_t)n);
    int32_t *it = xmalloc(sizeof(int32_t) * (size_t)n);
    for (int64_t j = 0; j < n; ++j) head[j] = -1;
    /* build child lists in ascending order by inserting descending at head */
    for (int64_t j = n - 1; j >= 0; --j)
        if (parent[j] != -1) {
            next[j] = head[parent[j]];
            head[parent[j]] = (int32_t)j;
        }
    int64_t k = 0;
    for (int64_t r = 0; r < n; ++r) {
        if (parent[r] != -1) continue;
        int64_t top = 0;
        stack[0] = (int32_t)r;
        it[r] = head[r];
        while (top >= 0) {
            int32_t v = stack[top];
            int32_t c = it[v];
            if (c != -1) {
                it[v] = next[c];
                stack[++top] = c;
                it[c] = head[c];
            } else {
                post[k++] = v;
                --top;
            }
        }
    }
    free(head);
    free(next);
    free(stack);
    free(it);
}

/*
 * orc_analyze: symbolic phase.
 *   n, colptr, rowidx : lower CSC of A including the diagonal, rows sorted
 *   perm              : fill-reducing order (perm[k] = original index)
 *   z                 : amalgamation tolerance (0 = fundamental supernodes)
 * Returns NULL when the input fails the basic checks.
 */
orc_sym *orc_analyze(int64_t n, const int64_t *colptr, const int32_t *rowidx,
                     const int32_t *perm_in, double z) {
    if (n < 0 || !colptr || (n > 0 && (!rowidx || !perm_in))) return NULL;
    for (int64_t c = 0; c < n; ++c)
        for (int64_t k = colptr[c]; k < colptr[c + 1]; ++k)
            if (rowidx[k] < c || rowidx[k] >= n) return NULL;
    orc_sym *S = xcalloc(1, sizeof(orc_sym));
    S->n = n;
    int32_t *iperm0 = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t k = 0; k < n; ++k) iperm0[perm_in[k]] = (int32_t)k;

    /* pass 1: etree of A(perm, perm), then its postorder */
    int64_t *Ap, *Amap;
    int32_t *Ai;
    permute_lower(n, colptr, rowidx, iperm0, &Ap, &Ai, &Amap);
    int32_t *parent0 = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    int64_t *Lp0;
    int32_t *Li0;
    column_merge(n, Ap, Ai, parent0, &Lp0, &Li0);
    S->post = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    postorder(n, parent0, S->post);
    free(Ap); free(Ai); free(Amap); free(parent0); free(Lp0); free(Li0);

    /* pass 2: the postordered matrix */
    S->perm = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    S->iperm = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int64_t k = 0; k < n; ++k) S->perm[k] = perm_in[S->post[k]];
    for (int64_t k = 0; k < n; ++k) S->iperm[S->perm[k]] = (int32_t)k;
    free(iperm0);
    permute_lower(n, colptr, rowidx, S->iperm, &S->Ap, &S->Ai, &S->Amap);
    S->parent = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    column_merge(n, S->Ap, S->Ai, S->parent, &S->Lp, &S->Li);
    S->colcount = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    S->flops = 0;
    S->nnzL = 0;
    for (int64_t j = 0; j < n; ++j) {
        int64_t c = S->Lp[j + 1] - S->Lp[j] + 1;
        S->colcount[j] = (int32_t)c;
        S->flops += c * c;
        S->nnzL += c;
    }

    /* fundamental supernodes: j+1 joins j's supernode iff parent(j) = j+1,
     * j+1 has exactly one child, and c_j = c_{j+1} + 1 */
    int32_t *nchild = xcalloc((size_t)n + 1, sizeof(int32_t));
    for (int64_t j = 0; j < n; ++j)
        if (S->parent[j] != -1) nchild[S->parent[j]]++;
    S->fund_ptr = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t nf = 0;
    for (int64_t j = 0; j < n; ++j) {
        int merge = j > 0 && S->parent[j - 1] == j && nchild[j] == 1 &&
                    S->colcount[j - 1] == S->colcount[j] + 1;
        if (!merge) S->fund_ptr[nf++] = (int32_t)j;
    }
    S->fund_ptr[nf] = (int32_t)n;
    S->nfund = nf;
    free(nchild);

    /* supernodal parent of each fundamental supernode */
    int32_t *fsn = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int32_t p = 0; p < nf; ++p)
        for (int32_t j = S->fund_ptr[p]; j < S->fund_ptr[p + 1]; ++j) fsn[j] = p;
    int32_t *fpar = xmalloc(sizeof(int32_t) * (size_t)(nf + 1));
    for (int32_t p = 0; p < nf; ++p) {
        int32_t last = S->fund_ptr[p + 1] - 1;
        fpar[p] = S->parent[last] == -1 ? -1 : fsn[S->parent[last]];
    }

    /* chain amalgamation: scan fundamental supernodes ascending; p joins the
     * group G that ends in p-1 iff fpar(p-1) = p and the merged group keeps
     * explicit zeros Z' within z of its stored entries E'.  For G of width W,
     * rows M, zeros Z and p of width w with |R_p| = m:
     *     W' = W + w, M' = W + m, Z' = Z + W (M' - M), E' = W'M' - W'(W'-1)/2
     * accepted iff (double)Z' <= z * (double)E'. */
    S->super_ptr = xmalloc(sizeof(int32_t) * (size_t)(nf + 1));
    int32_t *group_last = xmalloc(sizeof(int32_t) * (size_t)(nf + 1));
    int32_t ns = 0;
    int64_t W = 0, M = 0, Z = 0;
    S->zeros = 0;
    for (int32_t p = 0; p < nf; ++p) {
        int64_t w = S->fund_ptr[p + 1] - S->fund_ptr[p];
        int64_t m = S->colcount[S->fund_ptr[p]];
        int accept = 0;
        int64_t W2 = 0, M2 = 0, Z2 = 0;
        if (p > 0 && fpar[p - 1] == p) {
            W2 = W + w;
            M2 = W + m;
            Z2 = Z + W * (M2 - M);
            int64_t E2 = W2 * M2 - W2 * (W2 - 1) / 2;
            accept = (double)Z2 <= z * (double)E2;
        }
        if (accept) {
            W = W2; M = M2; Z = Z2;
            group_last[ns - 1] = p;
        } else {
            if (ns > 0) S->zeros += Z;
            S->super_ptr[ns] = S->fund_ptr[p];
            group_last[ns] = p;
            ns++;
            W = w; M = m; Z = 0;
        }
    }
    if (ns > 0) S->zeros += Z;
    S->super_ptr[ns] = (int32_t)n;
    S->nsuper = ns;

    S->snode = xmalloc(sizeof(int32_t) * (size_t)(n + 1));
    for (int32_t s = 0; s < ns; ++s)
        for (int32_t j = S->super_ptr[s]; j < S->super_ptr[s + 1]; ++j) S->snode[j] = s;
    S->sparent = xmalloc(sizeof(int32_t) * (size_t)(ns + 1));
    for (int32_t s = 0; s < ns; ++s) {
        int32_t last = S->super_ptr[s + 1] - 1;
        S->sparent[s] = S->parent[last] == -1 ? -1 : S->snode[S->parent[last]];
    }

    /* R_s = cols(s) U R_p, p the last fundamental supernode of the group;
     * R_p = {f_p} U S_{f_p} */
    S->rptr = xmalloc(sizeof(int64_t) * (size_t)(ns + 1));
    S->rptr[0] = 0;
    for (int32_t s = 0; s < ns; ++s) {
        int32_t p = group_last[s];
        int64_t cols_before = S->fund_ptr[p] - S->super_ptr[s];
        S->rptr[s + 1] = S->rptr[s] + cols_before + S->colcount[S->fund_ptr[p]];
    }
    S->rows = xmalloc(sizeof(int32_t) * (size_t)(S->rptr[ns] + 1));
    for (int32_t s = 0; s < ns; ++s) {
        int32_t p = group_last[s];
        int64_t o = S->rptr[s];
        for (int32_t j = S->super_ptr[s]; j < S->fund_ptr[p]; ++j) S->rows[o++] = j;
        int32_t fp = S->fund_ptr[p];
        S->rows[o++] = fp;
        for (int64_t k = S->Lp[fp]; k < S->Lp[fp + 1]; ++k) S->rows[o++] = S->Li[k];
    }
    free(group_last);
    free(fsn);
    free(fpar);

    S->lptr = xmalloc(sizeof(int64_t) * (size_t)(ns + 1));
    S->lptr[0] = 0;
    for (int32_t s = 0; s < ns; ++s) {
        int64_t m = S->rptr[s + 1] - S->rptr[s];
        int64_t w = S->super_ptr[s + 1] - S->super_ptr[s];
        S->lptr[s + 1] = S->lptr[s] + m * w;
    }

    /* U_s: every d < s with a row of R_d among cols(s), ascending in d */
    int64_t *ucnt = xcalloc((size_t)ns + 1, sizeof(int64_t));
    int32_t *last = xmalloc(sizeof(int32_t) * (size_t)(ns + 1));
    for (int32_t s = 0; s < ns; ++s) last[s] = -1;
    for (int32_t d = 0; d < ns; ++d)
        for (int64_t k = S->rptr[d]; k < S->rptr[d + 1]; ++k) {
            int32_t t = S->snode[S->rows[k]];
            if (t != d && last[t] != d) {
                last[t] = d;
                ucnt[t + 1]++;
            }
        }
    for (int32_t s = 0; s < ns; ++s) ucnt[s + 1] += ucnt[s];
    S->uptr = ucnt;
    S->ulist = xmalloc(sizeof(int32_t) * (size_t)(ucnt[ns] + 1));
    int64_t *cur = xmalloc(sizeof(int64_t) * (size_t)(ns + 1));
    for (int32_t s = 0; s < ns; ++s) { cur[s] = ucnt[s]; last[s] = -1; }
    for (int32_t d = 0; d < ns; ++d)
        for (int64_t k = S->rptr[d]; k < S->rptr[d + 1]; ++k) {
            int32_t t = S->snode[S->rows[k]];
            if (t != d && last[t] != d) {
                last[t] = d;
                S->ulist[cur[t]++] = d;
            }
        }
    free(cur);
    free(last);

    /* levels: children precede parents in a postorder, so one ascending pass */
    S->level = xcalloc((size_t)ns + 1, sizeof(int32_t));
    S->nlevels = ns > 0 ? 1 : 0;
    for (int32_t s = 0; s < ns; ++s) {
        int32_t p = S->sparent[s];
        if (p != -1 && S->level[p] < S->level[s] + 1) S->level[p] = S->level[s] + 1;
        if (S->level[s] + 1 > S->nlevels) S->nlevels = S->level[s] + 1;
    }
    return S;
}

void orc_free(orc_sym *S) {
    if (!S) return;
    free(S->perm); free(S->iperm); free(S->post); free(S->parent); free(S->colcount);
    free(S->Lp); free(S->Li); free(S->Ap); free(S->Ai); free(S->Amap); free(S->fund_ptr);
    free(S->super_ptr); free(S->snode); free(S->sparent); free(S->rptr); free(S->rows);
    free(S->lptr); free(S->uptr); free(S->ulist); free(S->level);
    free(S);
}

/* sizes[]: n, nsuper, nfund, sum|R_s|, panel entries, flops, nnzL, nlevels,
 *          sum|U_s|, explicit zeros */
void orc_sizes(const orc_sym *S, int64_t *out) {
    out[0] = S->n;
    out[1] = S->nsuper;
    out[2] = S->nfund;
    out[3] = S->rptr[S->nsuper];
    out[4] = S->lptr[S->nsuper];
    out[5] = S->flops;
    out[6] = S->nnzL;
    out[7] = S->nlevels;
    out[8] = S->uptr[S->nsuper];
    out[9] = S->zeros;
}

/* Copy one symbolic array out.  which: 0 perm, 1 parent, 2 colcount,
 * 3 super_ptr, 4 sparent, 5 rptr(int64), 6 rows, 7 lptr(int64), 8 uptr(int64),
 * 9 ulist, 10 level, 11 post, 12 Lp(int64), 13 Li, 14 fund_ptr */
int orc_get(const orc_sym *S, int which, void *dst) {
    int64_t n = S->n, ns = S->nsuper;
    switch (which) {
    case 0: memcpy(dst, S->perm, sizeof(int32_t) * (size_t)n); return 0;
    case 1: memcpy(dst, S->parent, sizeof(int32_t) * (size_t)n); return 0;
    case 2: memcpy(dst, S->colcount, sizeof(int32_t) * (size_t)n); return 0;
    case 3: memcpy(dst, S->super_ptr, sizeof(int32_t) * (size_t)(ns + 1)); return 0;
    case 4: memcpy(dst, S->sparent, sizeof(int32_t) * (size_t)ns); return 0;
    case 5: memcpy(dst, S->rptr, sizeof(int64_t) * (size_t)(ns + 1)); return 0;
    case 6: memcpy(dst, S->rows, sizeof(int32_t) * (size_t)S->rptr[ns]); return 0;
    case 7: memcpy(dst, S->lptr, sizeof(int64_t) * (size_t)(ns + 1)); return 0;
    case 8: memcpy(dst, S->uptr, sizeof(int64_t) * (size_t)(ns + 1)); return 0;
    case 9: memcpy(dst, S->ulist, sizeof(int32_t) * (size_t)S->uptr[ns]); return 0;
    case 10: memcpy(dst, S->level, sizeof(int32_t) * (size_t)ns); return 0;
    case 11: memcpy(dst, S->post, sizeof(int32_t) * (size_t)n); return 0;
    case 12: memcpy(dst, S->Lp, sizeof(int64_t) * (size_t)(n + 1)); return 0;
    case 13: memcpy(dst, S->Li, sizeof(int32_t) * (size_t)S->Lp[n]); return 0;
    case 14: memcpy(dst, S->fund_ptr, sizeof(int32_t) * (size_t)(S->nfund + 1)); return 0;
    default: return -1;
    }
}

/*
 * Left-looking step for one supernode s (Sec. 3, Listing 1): build it from A,
 * apply the update of every earlier supernode in U_s, then POTRF + TRSM.
 * Lx receives the column-major panel; Lr is a row-major mirror of the same
 * panels (entry (i, c) of supernode s at lptr[s] + i*w_s + c) so that every
 * inner product below walks contiguous memory.  The mirror changes no
 * arithmetic: each sum still runs over k in ascending order.  pos is n+1
 * ints of scratch.  Returns 0, or -2 with *bad_col set.
 */
static int factor_one(const orc_sym *S, const double *values, double *Lx, double *Lr, int32_t s,
                      int32_t *pos, int64_t *bad_col) {
    int32_t f = S->super_ptr[s], l = S->super_ptr[s + 1] - 1;
    int64_t w = l - f + 1, m = S->rptr[s + 1] - S->rptr[s];
    const int32_t *R = S->rows + S->rptr[s];
    double *B = Lr + S->lptr[s]; /* row-major m x w */
    for (int64_t k = 0; k < m; ++k) pos[R[k]] = (int32_t)k;
    /* construction of the supernode from A */
    memset(B, 0, sizeof(double) * (size_t)(m * w));
    for (int32_t j = f; j <= l; ++j)
        for (int64_t k = S->Ap[j]; k < S->Ap[j + 1]; ++k)
            B[(int64_t)pos[S->Ai[k]] * w + (j - f)] = values[S->Amap[k]];
    /* updates from every earlier supernode d that touches cols(s):
     * B[rel(R_d[r]), rel(R_d[c])] -= sum_k L_d[r,k] L_d[c,k],
     * for c in [i0, i1) (the rows of R_d inside cols(s)) and r >= c */
    for (int64_t u = S->uptr[s]; u < S->uptr[s + 1]; ++u) {
        int32_t d = S->ulist[u];
        int64_t md = S->rptr[d + 1] - S->rptr[d];
        int64_t wd = S->super_ptr[d + 1] - S->super_ptr[d];
        const int32_t *Rd = S->rows + S->rptr[d];
        const double *Ld = Lr + S->lptr[d];
        int64_t i0 = 0, i1;
        while (i0 < md && Rd[i0] < f) ++i0;
        i1 = i0;
        while (i1 < md && Rd[i1] <= l) ++i1;
        for (int64_t c = i0; c < i1; ++c) {
            int64_t col = Rd[c] - f;
            const double *lc = Ld + c * wd;
            for (int64_t r = c; r < md; ++r) {
                const double *lr = Ld + r * wd;
                double sum = 0.0;
                for (int64_t k = 0; k < wd; ++k) sum += lr[k] * lc[k];
                B[(int64_t)pos[Rd[r]] * w + col] -= sum;
            }
        }
    }
    /* column Cholesky of the diagonal block (POTRF) and of the rows
     * below it (TRSM by forward substitution):
     *   d    = b_jj - sum_{k<j} l_jk^2,  NOT_SPD unless d > 0 and finite
     *   l_jj = sqrt(d),  l_ij = (b_ij - sum_{k<j} l_ik l_jk) / l_jj */
    for (int64_t j = 0; j < w; ++j) {
        const double *lj = B + j * w;
        double d = lj[j];
        for (int64_t k = 0; k < j; ++k) d -= lj[k] * lj[k];
        if (!(d > 0.0) || !isfinite(d)) {
            if (bad_col) *bad_col = f + j;
            return -2;
        }
        double ljj = sqrt(d);
        B[j * w + j] = ljj;
        for (int64_t i = j + 1; i < m; ++i) {
            double *li = B + i * w;
            double v = li[j];
            for (int64_t k = 0; k < j; ++k) v -= li[k] * lj[k];
            li[j] = v / ljj;
        }
    }
    /* strict upper triangle of the diagonal block is not part of L */
    for (int64_t i = 0; i < w; ++i)
        for (int64_t c = i + 1; c < w; ++c) B[i * w + c] = 0.0;
    double *C = Lx + S->lptr[s];
    for (int64_t c = 0; c < w; ++c)
        for (int64_t i = 0; i < m; ++i) C[c * m + i] = B[i * w + c];
    return 0;
}

/* The left-looking loop over supernodes s_lo..s_hi in ascending order. */
static int factor_range(const orc_sym *S, const double *values, double *Lx, double *Lr,
                        int32_t s_lo, int32_t s_hi, int64_t *bad_col) {
    int32_t *pos = xmalloc(sizeof(int32_t) * (size_t)(S->n + 1));
    int rc = 0;
    if (bad_col) *bad_col = -1;
    for (int32_t s = s_lo; s <= s_hi && rc == 0; ++s) rc = factor_one(S, values, Lx, Lr, s, pos, bad_col);
    free(pos);
    return rc;
}

/*
 * orc_factor: left-looking supernodal numeric factorization.
 *   values : A's entries in the caller's CSC order
 *   Lx     : output, lptr[nsuper] doubles; supernode s is an m_s x w_s
 *            column-major block (leading dimension m_s) whose row k is global
 *            row rows[rptr[s]+k]; the strict upper triangle of each diagonal
 *            block is zero.
 * Returns 0, or -2 when a pivot is not positive (or not finite); *bad_col is
 * then the permuted index of that column (and -1 on success).
 */
int orc_factor(const orc_sym *S, const double *values, double *Lx, int64_t *bad_col) {
    double *Lr = xmalloc(sizeof(double) * (size_t)(S->lptr[S->nsuper] + 1));
    int rc = factor_range(S, values, Lx, Lr, 0, S->nsuper - 1, bad_col);
    free(Lr);
    return rc;
}

/*
 * orc_factor_parallel: the same factorization on `nthreads` host threads
 * (OpenMP), each thread owning whole supernodes, in the order of the
 * elimination tree: level by level (a supernode's level exceeds those of all
 * its descendants, which are all the supernodes its updates come from, Sec. 3
 * and Fig. 1).  This is the paper's one-task-per-supernode scheme without
 * nested tasks (NONESTED, Sec. 3-4).  Every supernode runs exactly the steps
 * of the sequential loop on the same inputs, so the result is bit-identical
 * to orc_factor for any thread count.  A supernode with a failed descendant
 * is skipped; the failure reported is the one of the lowest supernode, the
 * one the sequential loop stops at.  Returns the thread count used in
 * *used (nullable).  With roots (nroots of them) only the subtrees of those
 * supernodes are factored (a forest whose panels equal those of the whole
 * factorization, as in orc_factor_subtree); roots == NULL: all supernodes.
 */
static int32_t subtree_first(const orc_sym *S, int32_t root);

int orc_factor_parallel(const orc_sym *S, const double *values, double *Lx, int64_t *bad_col, int nthreads,
                        int *used, const int32_t *roots, int32_t nroots) {
    int32_t ns = S->nsuper;
    char *active = xcalloc((size_t)ns + 1, 1);
    if (roots) {
        for (int32_t q = 0; q < nroots; ++q) {
            if (roots[q] < 0 || roots[q] >= ns) { free(active); return -1; }
            for (int32_t t = subtree_first(S, roots[q]); t <= roots[q]; ++t) active[t] = 1;
        }
    } else {
        memset(active, 1, (size_t)ns);
    }
    double *Lr = xmalloc(sizeof(double) * (size_t)(S->lptr[ns] + 1));
    /* supernodes grouped by level */
    int32_t nl = S->nlevels;
    int64_t *lptr = xcalloc((size_t)nl + 2, sizeof(int64_t));
    int32_t *bylev = xmalloc(sizeof(int32_t) * (size_t)(ns + 1));
    for (int32_t s = 0; s < ns; ++s) lptr[S->level[s] + 1]++;
    for (int32_t v = 0; v < nl; ++v) lptr[v + 1] += lptr[v];
    {
        int64_t *fill = xmalloc(sizeof(int64_t) * (size_t)(nl + 1));
        for (int32_t v = 0; v <= nl; ++v) fill[v] = lptr[v];
        for (int32_t s = 0; s < ns; ++s) bylev[fill[S->level[s]]++] = s;
        free(fill);
    }
    /* failed[s]: s or one of its descendants failed */
    char *failed = xcalloc((size_t)ns + 1, 1);
    int64_t *badc = xmalloc(sizeof(int64_t) * (size_t)(ns + 1));
    int nt = nthreads > 0 ? nthreads : 1, got = 1;
    for (int32_t v = 0; v < nl; ++v) {
#pragma omp parallel num_threads(nt)
        {
#pragma omp single
            got = omp_get_num_threads_or_one();
            int32_t *pos = xmalloc(sizeof(int32_t) * (size_t)(S->n + 1));
#pragma omp for schedule(dynamic, 1)
            for (int64_t q = lptr[v]; q < lptr[v + 1]; ++q) {
                int32_t s = bylev[q];
                if (failed[s] || !active[s]) continue;
                int64_t bc = -1;
                if (factor_one(S, values, Lx, Lr, s, pos, &bc) != 0) {
                    failed[s] = 2; /* the supernode itself failed */
                    badc[s] = bc;
                }
            }
            free(pos);
        }
        /* a failure makes every ancestor skip */
        for (int64_t q = lptr[v]; q < lptr[v + 1]; ++q) {
            int32_t s = bylev[q], p = S->sparent[s];
            if (failed[s] && p >= 0 && !failed[p]) failed[p] = 1;
        }
    }
    int rc = 0;
    if (bad_col) *bad_col = -1;
    for (int32_t s = 0; s < ns; ++s)
        if (failed[s] == 2) {
            rc = -2;
            if (bad_col) *bad_col = badc[s];
            break;
        }
    if (used) *used = got;
    free(failed); free(badc); free(bylev); free(lptr); free(Lr); free(active);
    return rc;
}

/* First supernode of the subtree of `root` (its descendants and itself are a
 * contiguous range in postorder): walk down while the supernode just below
 * the range still descends from root. */
static int32_t subtree_first(const orc_sym *S, int32_t root) {
    int32_t lo = root;
    for (int32_t s = root - 1; s >= 0; --s) {
        int32_t a = s;
        while (a != -1 && a < root) a = S->sparent[a];
        if (a != root) break;
        lo = s;
    }
    return lo;
}

/*
 * orc_factor_subtree: the same factorization restricted to the subtree of
 * supernode `root` (its descendants and itself, a contiguous range in
 * postorder).  Left-looking updates into a supernode come only from its
 * descendants, so these panels equal those of the full factorization; the
 * other panels of Lx are left untouched.  *first receives the first supernode
 * of the range.
 */
int orc_factor_subtree(const orc_sym *S, const double *values, int32_t root, double *Lx,
                       int64_t *bad_col, int32_t *first) {
    if (root < 0 || root >= S->nsuper) return -1;
    int32_t lo = subtree_first(S, root);
    if (first) *first = lo;
    double *Lr = xmalloc(sizeof(double) * (size_t)(S->lptr[S->nsuper] + 1));
    int rc = factor_range(S, values, Lx, Lr, lo, root, bad_col);
    free(Lr);
    return rc;
}

/*
 * orc_solve: X := A^{-1} X for nrhs right-hand sides (column-major, leading
 * dimension ldb, original ordering) using a factor from orc_factor.
 */
void orc_solve(const orc_sym *S, const double *Lx, double *X, int64_t nrhs, int64_t ldb) {
    int64_t n = S->n;
    int32_t ns = S->nsuper;
    double *b = xmalloc(sizeof(double) * (size_t)(n + 1));
    for (int64_t r = 0; r < nrhs; ++r) {
        double *x = X + r * ldb;
        for (int64_t k = 0; k < n; ++k) b[k] = x[S->perm[k]];
        /* forward: L y = b */
        for (int32_t s = 0; s < ns; ++s) {
            int32_t f = S->super_ptr[s];
            int64_t w = S->super_ptr[s + 1] - f, m = S->rptr[s + 1] - S->rptr[s];
            const int32_t *R = S->rows + S->rptr[s];
            const double *L = Lx + S->lptr[s];
            for (int64_t j = 0; j < w; ++j) {
                double v = b[f + j];
                for (int64_t k = 0; k < j; ++k) v -= L[k * m + j] * b[f + k];
                b[f + j] = v / L[j * m + j];
            }
            for (int64_t i = w; i < m; ++i) {
                double v = 0.0;
                for (int64_t k = 0; k < w; ++k) v += L[k * m + i] * b[f + k];
                b[R[i]] -= v;
            }
        }
        /* backward: L^T x = y */
        for (int32_t s = ns - 1; s >= 0; --s) {
            int32_t f = S->super_ptr[s];
            int64_t w = S->super_ptr[s + 1] - f, m = S->rptr[s + 1] - S->rptr[s];
            const int32_t *R = S->rows + S->rptr[s];
            const double *L = Lx + S->lptr[s];
            for (int64_t k = 0; k < w; ++k) {
                double v = 0.0;
                for (int64_t i = w; i < m; ++i) v += L[k * m + i] * b[R[i]];
                b[f + k] -= v;
            }
            for (int64_t j = w - 1; j >= 0; --j) {
                double v = b[f + j];
                for (int64_t k = j + 1; k < w; ++k) v -= L[j * m + k] * b[f + k];
                b[f + j] = v / L[j * m + j];
            }
        }
        for (int64_t k = 0; k < n; ++k) x[S->perm[k]] = b[k];
    }
    free(b);
}
