// The paper's comparison orderings of the single-SpMxV framework (Section
// 5.1): sBFS and sRCM work on the bipartite graph of A, whose vertices are
// the m rows and the n columns and whose edges are the nonzeros; the visit
// order of the row vertices gives the row order and that of the column
// vertices the column order.
//
// Vertex numbering: row i is vertex i, column j is vertex m + j.  The paper
// leaves the start vertices and tie-breaks open; the readings here:
//  * sBFS: components in order of their smallest vertex; breadth-first
//    search from that vertex, neighbours in increasing vertex number.
//  * sRCM: reverse Cuthill-McKee; components in order of their smallest
//    vertex; each starts at a pseudo-peripheral vertex found by George and
//    Liu's search from the component's vertex of least degree (smallest
//    number on ties): repeat a breadth-first search from the current start
//    and move to the least-degree vertex of its last level (smallest number
//    on ties) while that raises the eccentricity.  Cuthill-McKee then visits
//    the unvisited neighbours of each vertex by increasing degree (number on
//    ties); the whole visit sequence is reversed at the end.
#include <algorithm>
#include <memory>
#include <string>
#include <vector>

#include "api_internal.h"

using namespace spx;

namespace {

struct Bipartite {
    int32_t m = 0, n = 0;
    std::vector<int64_t> off;  // [m + n + 1]
    std::vector<int32_t> adj;  // neighbours of every vertex, ascending
    int32_t nv() const { return m + n; }
    int64_t deg(int32_t v) const { return off[v + 1] - off[v]; }
};

Bipartite bipartite_of(const CsrHost &A) {
    Bipartite G;
    G.m = A.m;
    G.n = A.n;
    const int32_t nv = A.m + A.n;
    G.off.assign((size_t)nv + 1, 0);
    for (int32_t i = 0; i < A.m; ++i) G.off[i + 1] = A.rowptr[i + 1] - A.rowptr[i];
    for (int64_t q = 0; q < A.nnz; ++q) G.off[A.m + A.colidx[q] + 1]++;
    for (int32_t v = 0; v < nv; ++v) G.off[v + 1] += G.off[v];
    G.adj.resize((size_t)G.off[nv]);
    std::vector<int64_t> fill(G.off.begin(), G.off.end() - 1);
    // rows list their columns ascending (CSR order); columns list their
    // rows ascending because rows are scanned in order
    for (int32_t i = 0; i < A.m; ++i)
        for (int32_t q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
            const int32_t c = A.m + A.colidx[q];
            G.adj[fill[i]++] = c;
            G.adj[fill[c]++] = i;
        }
    return G;
}

// Breadth-first search from `start` over the vertices not yet marked with
// `stamp` (neighbours in adjacency order): returns the visit order;
// `last_level` receives the vertices of the deepest level and `levels` the
// number of levels.
std::vector<int32_t> bfs_levels(const Bipartite &G, int32_t start, std::vector<int32_t> &mark, int32_t stamp,
                                std::vector<int32_t> &last_level, int32_t *levels = nullptr) {
    std::vector<int32_t> order{start};
    mark[start] = stamp;
    size_t lo = 0;
    int32_t nlev = 0;
    last_level.assign(1, start);
    while (lo < order.size()) {
        const size_t hi = order.size();
        for (size_t t = lo; t < hi; ++t)
            for (int64_t e = G.off[order[t]]; e < G.off[order[t] + 1]; ++e) {
                const int32_t w = G.adj[e];
                if (mark[w] != stamp) {
                    mark[w] = stamp;
                    order.push_back(w);
                }
            }
        ++nlev;
        if (order.size() > hi) last_level.assign(order.begin() + hi, order.end());
        lo = hi;
    }
    if (levels) *levels = nlev;
    return order;
}

void split_order(const Bipartite &G, const std::vector<int32_t> &seq, int32_t *row_perm, int32_t *col_perm) {
    int32_t r = 0, c = 0;
    for (int32_t v : seq) {
        if (v < G.m) row_perm[r++] = v;
        else col_perm[c++] = v - G.m;
    }
}

}  // namespace

namespace spx {

void order_bfs(const CsrHost &A, int32_t *row_perm, int32_t *col_perm) {
    const Bipartite G = bipartite_of(A);
    std::vector<int32_t> mark(G.nv(), -1), seq, lvl;
    seq.reserve(G.nv());
    for (int32_t v = 0; v < G.nv(); ++v) {
        if (mark[v] >= 0) continue;
        std::vector<int32_t> part = bfs_levels(G, v, mark, 0, lvl);
        seq.insert(seq.end(), part.begin(), part.end());
    }
    split_order(G, seq, row_perm, col_perm);
}

void order_rcm(const CsrHost &A, int32_t *row_perm, int32_t *col_perm) {
    const Bipartite G = bipartite_of(A);
    const int32_t nv = G.nv();
    std::vector<int32_t> done(nv, 0), mark(nv, -1), seq, lvl, comp;
    seq.reserve(nv);
    int32_t stamp = 0;
    for (int32_t v0 = 0; v0 < nv; ++v0) {
        if (done[v0]) continue;
        // the component of v0 and its least-degree vertex
        comp = bfs_levels(G, v0, mark, stamp++, lvl);
        int32_t start = comp[0];
        for (int32_t w : comp)
            if (G.deg(w) < G.deg(start) || (G.deg(w) == G.deg(start) && w < start)) start = w;
        // George and Liu's pseudo-peripheral vertex
        int32_t ecc = 0;
        bfs_levels(G, start, mark, stamp++, lvl, &ecc);
        for (;;) {
            int32_t cand = lvl[0];
            for (int32_t w : lvl)
                if (G.deg(w) < G.deg(cand) || (G.deg(w) == G.deg(cand) && w < cand)) cand = w;
            std::vector<int32_t> lvl2;
            int32_t e2 = 0;
            bfs_levels(G, cand, mark, stamp++, lvl2, &e2);
            if (e2 <= ecc) break;
            start = cand;
            ecc = e2;
            lvl.swap(lvl2);
        }
        // Cuthill-McKee from start
        const size_t base = seq.size();
        seq.push_back(start);
        done[start] = 1;
        std::vector<int32_t> nb;
        for (size_t t = base; t < seq.size(); ++t) {
            nb.clear();
            for (int64_t e = G.off[seq[t]]; e < G.off[seq[t] + 1]; ++e)
                if (!done[G.adj[e]]) nb.push_back(G.adj[e]);
            std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) {
                return G.deg(a) != G.deg(b) ? G.deg(a) < G.deg(b) : a < b;
            });
            for (int32_t w : nb) {
                done[w] = 1;
                seq.push_back(w);
            }
        }
    }
    std::reverse(seq.begin(), seq.end());
    split_order(G, seq, row_perm, col_perm);
}

}  // namespace spx

namespace {

void check_bijection(const int32_t *p, int32_t n, const char *what) {
    std::vector<uint8_t> seen(n, 0);
    for (int32_t i = 0; i < n; ++i) {
        if (p[i] < 0 || p[i] >= n || seen[p[i]]) fail(SPX_EINVAL, std::string(what) + " is not a permutation");
        seen[p[i]] = 1;
    }
}

}  // namespace

extern "C" {

spx_status spx_order_bfs(spx_mat A, int32_t *row_perm, int32_t *col_perm) {
    return guarded([&] {
        if (!A || (A->h.m && !row_perm) || (A->h.n && !col_perm)) fail(SPX_EINVAL, "NULL argument");
        order_bfs(A->h, row_perm, col_perm);
    });
}

spx_status spx_order_rcm(spx_mat A, int32_t *row_perm, int32_t *col_perm) {
    return guarded([&] {
        if (!A || (A->h.m && !row_perm) || (A->h.n && !col_perm)) fail(SPX_EINVAL, "NULL argument");
        order_rcm(A->h, row_perm, col_perm);
    });
}

spx_status spx_plan_from_perm(spx_mat A, const int32_t *row_perm, const int32_t *col_perm, const spx_tune *tune,
                              spx_plan *out) {
    return guarded([&] {
        if (!A || !out || (A->h.m && !row_perm) || (A->h.n && !col_perm)) fail(SPX_EINVAL, "NULL argument");
        *out = nullptr;
        check_bijection(row_perm, A->h.m, "row_perm");
        check_bijection(col_perm, A->h.n, "col_perm");
        std::unique_ptr<spx_plan_s> P(new spx_plan_s());
        plan_from_perm(*P, A->h, row_perm, col_perm);
        spx_tune t{};
        if (tune) t = *tune;
        if (t.window_entries == 0) t.window_entries = -1;
        P->tune = resolve_tune(&t, P->form);
        build_schedule(*P);
        upload_plan(*P, *A, nullptr);
        *out = P.release();
    });
}

}  // extern "C"
