// ordering.cpp -- fill-reducing orderings for input without coordinates
// (spc_order; the paper's Sec. 2 names METIS and AMD as the orderings
// CHOLMOD tries).  Two methods of this library's own:
//
//  - graph nested dissection by level structures (George's automatic nested
//    dissection): in each connected part, a breadth-first level structure
//    rooted at a pseudo-peripheral vertex; the separator is the level, among
//    those that leave both sides at least a third of the part, with the
//    fewest vertices, thinned to its vertices that touch the level above;
//    both sides are ordered recursively, then the separator.  Parts of at
//    most kLeaf vertices are ordered by minimum degree.
//  - minimum degree (Tinney-Walker / Rose): repeatedly eliminate a vertex
//    of least degree in the elimination graph, which becomes a clique of
//    its neighbours; exact degrees on an explicit graph, with ties broken by
//    the lowest index.  Quadratic in the worst case: meant for parts and
//    small matrices.
#include <algorithm>
#include <cstdint>
#include <numeric>
#include <queue>
#include <set>
#include <vector>

#include "plan.h"

namespace spc {
namespace {

constexpr int kLeaf = 64;
// whole-matrix minimum degree is refused above this order (its explicit
// elimination graph grows with the fill)
constexpr int64_t kMinDegreeMax = 10000;

struct Graph {
    int64_t n = 0;
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;  // symmetric, no self loops
};

// The symmetric adjacency of a lower-CSC pattern.
bool build_graph(int64_t n, const int64_t *colptr, const int32_t *rowidx, Graph &G) {
    G.n = n;
    G.ptr.assign(n + 1, 0);
    for (int64_t c = 0; c < n; ++c)
        for (int64_t k = colptr[c]; k < colptr[c + 1]; ++k) {
            const int64_t r = rowidx[k];
            if (r < c || r >= n) return false;
            if (r == c) continue;
            G.ptr[r + 1]++;
            G.ptr[c + 1]++;
        }
    for (int64_t i = 0; i < n; ++i) G.ptr[i + 1] += G.ptr[i];
    G.adj.resize(G.ptr[n]);
    std::vector<int64_t> fill(G.ptr.begin(), G.ptr.end() - 1);
    for (int64_t c = 0; c < n; ++c)
        for (int64_t k = colptr[c]; k < colptr[c + 1]; ++k) {
            const int32_t r = rowidx[k];
            if (r == c) continue;
            G.adj[fill[r]++] = (int32_t)c;
            G.adj[fill[c]++] = r;
        }
    return true;
}

// Minimum degree on the subgraph induced by `verts` (exact degrees on an
// explicit elimination graph); appends the order to `out`.
void min_degree(const Graph &G, const std::vector<int32_t> &verts, std::vector<int32_t> &out) {
    const int64_t m = (int64_t)verts.size();
    // local ids
    std::vector<std::pair<int32_t, int32_t>> idx;
    idx.reserve(m);
    for (int64_t i = 0; i < m; ++i) idx.push_back({verts[i], (int32_t)i});
    std::sort(idx.begin(), idx.end());
    auto local = [&](int32_t v) -> int32_t {
        auto it = std::lower_bound(idx.begin(), idx.end(), std::make_pair(v, -1));
        return (it != idx.end() && it->first == v) ? it->second : -1;
    };
    std::vector<std::set<int32_t>> nb(m);
    for (int64_t i = 0; i < m; ++i) {
        const int32_t v = verts[i];
        for (int64_t k = G.ptr[v]; k < G.ptr[v + 1]; ++k) {
            const int32_t u = local(G.adj[k]);
            if (u >= 0) nb[i].insert(u);
        }
    }
    std::set<std::pair<int64_t, int32_t>> byd;  // (degree, vertex)
    for (int64_t i = 0; i < m; ++i) byd.insert({(int64_t)nb[i].size(), (int32_t)i});
    std::vector<char> gone(m, 0);
    while (!byd.empty()) {
        const int32_t v = byd.begin()->second;
        byd.erase(byd.begin());
        gone[v] = 1;
        out.push_back(verts[v]);
        std::vector<int32_t> cl(nb[v].begin(), nb[v].end());
        for (int32_t u : cl) byd.erase({(int64_t)nb[u].size(), u});
        for (int32_t u : cl) {
            nb[u].erase(v);
            for (int32_t w : cl)
                if (w != u) nb[u].insert(w);
        }
        for (int32_t u : cl) byd.insert({(int64_t)nb[u].size(), u});
        nb[v].clear();
    }
}

// Breadth-first levels from `root` inside the vertices marked `mark[v] ==
// tag`; returns the levels (level[v]) and the order of visit.
int32_t bfs_levels(const Graph &G, int32_t root, const std::vector<int32_t> &mark, int32_t tag,
                   std::vector<int32_t> &level, std::vector<int32_t> &order) {
    order.clear();
    order.push_back(root);
    level[root] = 0;
    int32_t depth = 0;
    for (size_t h = 0; h < order.size(); ++h) {
        const int32_t v = order[h];
        for (int64_t k = G.ptr[v]; k < G.ptr[v + 1]; ++k) {
            const int32_t u = G.adj[k];
            if (mark[u] != tag || level[u] >= 0) continue;
            level[u] = level[v] + 1;
            depth = std::max(depth, level[u]);
            order.push_back(u);
        }
    }
    return depth;
}

struct NdState {
    const Graph &G;
    std::vector<int32_t> mark, level, order;
    int32_t next_tag = 1;
    std::vector<int32_t> out;
    explicit NdState(const Graph &g) : G(g), mark(g.n, 0), level(g.n, -1) {}
};

// Order the connected vertex set `part` (all marked `tag`): recursive
// dissection, appended to st.out.
void dissect(NdState &st, std::vector<int32_t> part, int32_t tag);

// Split `verts` (marked tag) into connected components and dissect each.
void components(NdState &st, const std::vector<int32_t> &verts, int32_t tag) {
    for (int32_t v : verts) st.level[v] = -1;
    for (int32_t v : verts) {
        if (st.level[v] >= 0) continue;
        bfs_levels(st.G, v, st.mark, tag, st.level, st.order);
        std::vector<int32_t> comp = st.order;
        const int32_t t = st.next_tag++;
        for (int32_t u : comp) st.mark[u] = t;
        dissect(st, std::move(comp), t);
    }
}

void dissect(NdState &st, std::vector<int32_t> part, int32_t tag) {
    if ((int64_t)part.size() <= kLeaf) {
        min_degree(st.G, part, st.out);
        return;
    }
    // pseudo-peripheral root: a farthest vertex, while the depth grows
    for (int32_t v : part) st.level[v] = -1;
    int32_t root = part[0];
    int32_t depth = bfs_levels(st.G, root, st.mark, tag, st.level, st.order);
    for (int it = 0; it < 4; ++it) {
        const int32_t far = st.order.back();
        for (int32_t v : part) st.level[v] = -1;
        const int32_t d2 = bfs_levels(st.G, far, st.mark, tag, st.level, st.order);
        if (d2 <= depth) {
            for (int32_t v : part) st.level[v] = -1;
            depth = bfs_levels(st.G, root, st.mark, tag, st.level, st.order);
            break;
        }
        root = far;
        depth = d2;
    }
    if (depth < 2) {  // (nearly) a clique: no level separates it
        min_degree(st.G, part, st.out);
        return;
    }
    // level sizes and cumulative counts; the separator level: fewest vertices
    // among those leaving at least a third of the part on each side
    std::vector<int64_t> cnt(depth + 1, 0);
    for (int32_t v : part) cnt[st.level[v]]++;
    const int64_t N = (int64_t)part.size();
    int64_t below = 0, best = -1, bestc = INT64_MAX;
    for (int32_t l = 0; l <= depth; ++l) {
        const int64_t above = N - below - cnt[l];
        if (l > 0 && l < depth && 3 * below >= N && 3 * above >= N && cnt[l] < bestc) {
            bestc = cnt[l];
            best = l;
        }
        below += cnt[l];
    }
    if (best < 0) {  // no balanced level: the middle one
        int64_t acc = 0;
        for (int32_t l = 0; l <= depth; ++l) {
            acc += cnt[l];
            if (2 * acc >= N) {
                best = std::max(1, std::min(depth - 1, l));
                break;
            }
        }
    }
    // separator: vertices of level `best` with a neighbour in level best + 1
    std::vector<int32_t> lo, hi, sep;
    for (int32_t v : part) {
        const int32_t l = st.level[v];
        if (l < best) {
            lo.push_back(v);
        } else if (l > best) {
            hi.push_back(v);
        } else {
            bool touches = false;
            for (int64_t k = st.G.ptr[v]; k < st.G.ptr[v + 1] && !touches; ++k) {
                const int32_t u = st.G.adj[k];
                touches = st.mark[u] == tag && st.level[u] == best + 1;
            }
            (touches ? sep : lo).push_back(v);
        }
    }
    const int32_t tlo = st.next_tag++, thi = st.next_tag++, tsep = st.next_tag++;
    for (int32_t v : lo) st.mark[v] = tlo;
    for (int32_t v : hi) st.mark[v] = thi;
    for (int32_t v : sep) st.mark[v] = tsep;
    components(st, lo, tlo);
    components(st, hi, thi);
    // the separator last (its own vertices by minimum degree)
    min_degree(st.G, sep, st.out);
}

}  // namespace

int order_graph(int64_t n, const int64_t *colptr, const int32_t *rowidx, int method, int32_t *perm) {
    Graph G;
    if (!build_graph(n, colptr, rowidx, G)) return -1;
    if (method == 0) {
        std::iota(perm, perm + n, 0);
        return 0;
    }
    std::vector<int32_t> all(n);
    std::iota(all.begin(), all.end(), 0);
    if (method == 2) {
        if (n > kMinDegreeMax) return -1;
        std::vector<int32_t> out;
        out.reserve(n);
        min_degree(G, all, out);
        std::copy(out.begin(), out.end(), perm);
        return 0;
    }
    if (method != 1) return -1;
    NdState st(G);
    st.out.reserve(n);
    for (int32_t v : all) st.mark[v] = 0;
    components(st, all, 0);
    if ((int64_t)st.out.size() != n) return -1;
    std::copy(st.out.begin(), st.out.end(), perm);
    return 0;
}

}  // namespace spc
