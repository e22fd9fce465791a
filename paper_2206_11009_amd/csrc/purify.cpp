// Purification of the final plan to a basic (acyclic) one (host C++).
//
// Section 2.2: the bipartite graph of any vertex of the transport polytope is
// acyclic, so an optimal plan with at most m+n-1 nonzeros exists; the
// interior-point iterate approaches a point of the (possibly degenerate)
// optimal face instead.  Every cycle of the support is cancelled by pushing
// flow around it in the direction that does not raise the cost until one of
// its edges empties; row and column sums are unchanged by such pushes.  Then
// flows below drop_rel * min(a_i, b_j) are taken as zero and the flows of the
// remaining forest are recomputed from the marginals by leaf elimination.
//
// The spanning forest is kept rooted (parent, parent edge, depth), so the
// cycle of a non-forest edge is found by climbing from both ends to their
// common ancestor, and an edge swap re-hangs only the detached subtree.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <functional>
#include <numeric>
#include <queue>
#include <vector>

namespace otip {

namespace {

struct DSU {
    std::vector<int> p;
    explicit DSU(int n) : p(n) { std::iota(p.begin(), p.end(), 0); }
    int find(int x) {
        while (p[x] != x) x = p[x] = p[p[x]];
        return x;
    }
    bool unite(int a, int b) {
        a = find(a);
        b = find(b);
        if (a == b) return false;
        p[a] = b;
        return true;
    }
};

struct Forest {
    int V;
    std::vector<std::vector<std::pair<int, int>>> adj;  // (node, edge)
    std::vector<char> in_forest;
    std::vector<int> parent, pedge, depth;

    Forest(int v, int E) : V(v), adj(v), in_forest(E, 0), parent(v, -1), pedge(v, -1), depth(v, 0) {}

    // remove edge e from the adjacency of node u (the lists hold forest edges
    // only, so that re-hanging a subtree walks the tree and nothing else)
    void unlink(int u, int e) {
        auto &L = adj[u];
        for (size_t q = 0; q < L.size(); ++q)
            if (L[q].second == e) {
                L[q] = L.back();
                L.pop_back();
                return;
            }
    }

    void hang(int root, int par, int pe, int d0) {
        // BFS over forest edges from root, parent pointers away from `par`
        std::queue<int> q;
        parent[root] = par;
        pedge[root] = pe;
        depth[root] = d0;
        q.push(root);
        while (!q.empty()) {
            const int u = q.front();
            q.pop();
            for (auto [v, e] : adj[u]) {
                if (!in_forest[e] || e == pedge[u]) continue;
                parent[v] = u;
                pedge[v] = e;
                depth[v] = depth[u] + 1;
                q.push(v);
            }
        }
    }
};

// The sign of an exact sum of doubles, so that the direction taken around a
// cycle does not depend on rounding (costs such as square roots are not
// integers).  The terms are accumulated into a nonoverlapping expansion with
// error-free additions (Knuth's two-sum), the grow-expansion of Shewchuk's
// adaptive-precision arithmetic with zero components dropped; the largest
// component of such an expansion has the sign of the sum.
struct ExactSum {
    std::vector<double> e;  // increasing magnitude, nonoverlapping
    void add(double b) {
        size_t k = 0;
        for (size_t q = 0; q < e.size(); ++q) {
            const double s = b + e[q];
            const double bv = s - b;
            const double err = (b - (s - bv)) + (e[q] - bv);
            if (err != 0.0) e[k++] = err;
            b = s;
        }
        e.resize(k);
        if (b != 0.0) e.push_back(b);
    }
    int sign() const { return e.empty() ? 0 : (e.back() > 0.0 ? 1 : -1); }
};

}  // namespace

// One purification attempt; returns true when the forest flows recomputed from
// the marginals are nonnegative (an exactly feasible basic plan).
static bool purify_attempt(int m, int n, const std::vector<int32_t> &rows_in,
                           const std::vector<int32_t> &cols_in, const std::vector<double> &flows_in,
                           const std::vector<double> &costs_in, const std::vector<double> &a,
                           const std::vector<double> &b, double drop_rel, bool predrop,
                           std::vector<int32_t> &orows, std::vector<int32_t> &ocols,
                           std::vector<double> &oflows) {
    std::vector<int32_t> R, C;
    std::vector<double> F;
    std::vector<double> W;
    // with predrop, numerically-zero flows leave before any cycle is cancelled
    for (size_t k = 0; k < flows_in.size(); ++k)
        if (flows_in[k] > 0.0 &&
            (!predrop || flows_in[k] >= drop_rel * std::min(a[rows_in[k]], b[cols_in[k]]))) {
            R.push_back(rows_in[k]);
            C.push_back(cols_in[k]);
            F.push_back(flows_in[k]);
            W.push_back(costs_in[k]);
        }
    const int E = (int)F.size();
    const int V = m + n;
    auto vidx = [&](int e) { return (uint64_t)R[e] + (uint64_t)C[e] * (uint64_t)m; };
    std::vector<int> order(E);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int x, int y) {
        if (F[x] != F[y]) return F[x] > F[y];
        return vidx(x) < vidx(y);
    });
    Forest fo(V, E);
    DSU dsu(V);
    std::vector<int> nonforest;
    for (int e : order) {
        const int u = R[e], v = m + C[e];
        if (dsu.unite(u, v)) {
            fo.in_forest[e] = 1;
            fo.adj[u].push_back({v, e});
            fo.adj[v].push_back({u, e});
        } else {
            nonforest.push_back(e);
        }
    }
    std::vector<char> seen(V, 0);
    for (int r = 0; r < V; ++r)
        if (fo.parent[r] < 0 && !seen[r]) {
            fo.hang(r, -1, -1, 0);
            // mark the component
            std::queue<int> q;
            q.push(r);
            seen[r] = 1;
            while (!q.empty()) {
                int u = q.front();
                q.pop();
                for (auto [v, e] : fo.adj[u])
                    if (fo.in_forest[e] && !seen[v]) {
                        seen[v] = 1;
                        q.push(v);
                    }
            }
        }
    std::vector<char> alive(E, 1);
    std::vector<int> up_u, up_v;
    for (int e : nonforest) {
        const int u = R[e], v = m + C[e];
        // forest path from v (column node) to u (row node): climb both sides
        up_u.clear();
        up_v.clear();
        int x = u, y = v;
        while (x != y) {
            if (fo.depth[x] >= fo.depth[y]) {
                up_u.push_back(fo.pedge[x]);
                x = fo.parent[x];
            } else {
                up_v.push_back(fo.pedge[y]);
                y = fo.parent[y];
            }
        }
        // path v -> lca -> u
        std::vector<int> path(up_v.begin(), up_v.end());
        path.insert(path.end(), up_u.rbegin(), up_u.rend());
        // alternate: 1st, 3rd, ... path edges decrease when e increases
        ExactSum dcost;
        dcost.add(W[e]);
        for (size_t t = 0; t < path.size(); ++t) dcost.add((t % 2 == 0) ? -W[path[t]] : W[path[t]]);
        // e increases only where that lowers the cost; on a tie it decreases,
        // and as the smallest flow on its cycle of the maximum-flow forest it
        // then usually leaves, so the forest is not re-hung
        std::vector<int> dec, inc;
        if (dcost.sign() < 0) {
            inc.push_back(e);
            for (size_t t = 0; t < path.size(); ++t) (t % 2 == 0 ? dec : inc).push_back(path[t]);
        } else {
            dec.push_back(e);
            for (size_t t = 0; t < path.size(); ++t) (t % 2 == 0 ? inc : dec).push_back(path[t]);
        }
        int bott = dec[0];
        for (int k : dec)
            if (F[k] < F[bott] || (F[k] == F[bott] && vidx(k) < vidx(bott))) bott = k;
        const double t = F[bott];
        for (int k : dec) F[k] -= t;
        for (int k : inc) F[k] += t;
        F[bott] = 0.0;
        alive[bott] = 0;
        if (bott != e) {
            // swap bott out of the forest and e in; re-hang the detached subtree
            const int bu = R[bott], bv = m + C[bott];
            const int child = (fo.parent[bu] == bv && fo.pedge[bu] == bott) ? bu : bv;
            fo.in_forest[bott] = 0;
            fo.in_forest[e] = 1;
            fo.unlink(bu, bott);
            fo.unlink(bv, bott);
            fo.adj[u].push_back({v, e});
            fo.adj[v].push_back({u, e});
            // which endpoint of e lies in the detached subtree of `child`?
            auto in_sub = [&](int z) {
                while (z >= 0 && fo.depth[z] > fo.depth[child]) z = fo.parent[z];
                return z == child;
            };
            const int w = in_sub(u) ? u : v;
            const int other = (w == u) ? v : u;
            fo.hang(w, other, e, fo.depth[other] + 1);
        }
    }
    // drop numerical zeros, then recompute the forest flows from the marginals
    std::vector<int> keep;
    for (int e = 0; e < E; ++e)
        if (alive[e] && F[e] > 0.0 && F[e] >= drop_rel * std::min(a[R[e]], b[C[e]])) keep.push_back(e);
    std::vector<double> rem(V);
    for (int i = 0; i < m; ++i) rem[i] = a[i];
    for (int j = 0; j < n; ++j) rem[m + j] = b[j];
    std::vector<std::vector<int>> inc(V);
    for (int e : keep) {
        inc[R[e]].push_back(e);
        inc[m + C[e]].push_back(e);
    }
    std::vector<int> deg(V);
    for (int q = 0; q < V; ++q) deg[q] = (int)inc[q].size();
    std::vector<char> used(E, 0);
    std::vector<double> exact(E, 0.0);
    std::priority_queue<int, std::vector<int>, std::greater<int>> leaves;
    for (int q = 0; q < V; ++q)
        if (deg[q] == 1) leaves.push(q);
    while (!leaves.empty()) {
        const int q = leaves.top();
        leaves.pop();
        if (deg[q] != 1) continue;
        int e = -1;
        for (int k : inc[q])
            if (!used[k]) {
                e = k;
                break;
            }
        used[e] = 1;
        const int o = (q < m) ? m + C[e] : R[e];
        exact[e] = rem[q];
        rem[q] = 0.0;
        rem[o] -= exact[e];
        deg[q] = 0;
        if (--deg[o] == 1) leaves.push(o);
    }
    double mn = 0.0, mx = 0.0;
    for (int e : keep) {
        mn = std::min(mn, exact[e]);
        mx = std::max(mx, exact[e]);
    }
    const bool use_exact = !keep.empty() && mn >= -1e-12 * mx;
    std::vector<int> out = use_exact ? keep : std::vector<int>();
    if (!use_exact)
        for (int e = 0; e < E; ++e)
            if (alive[e] && F[e] > 0.0) out.push_back(e);
    std::sort(out.begin(), out.end(), [&](int x, int y) { return vidx(x) < vidx(y); });
    orows.clear();
    ocols.clear();
    oflows.clear();
    for (int e : out) {
        const double f = use_exact ? std::max(exact[e], 0.0) : F[e];
        orows.push_back(R[e]);
        ocols.push_back(C[e]);
        oflows.push_back(f);
    }
    return use_exact;
}

void purify_plan(int m, int n, const std::vector<int32_t> &rows_in,
                 const std::vector<int32_t> &cols_in, const std::vector<double> &flows_in,
                 const std::vector<double> &costs_in, const std::vector<double> &a,
                 const std::vector<double> &b, double drop_rel, std::vector<int32_t> &orows,
                 std::vector<int32_t> &ocols, std::vector<double> &oflows) {
    if (purify_attempt(m, n, rows_in, cols_in, flows_in, costs_in, a, b, drop_rel, true, orows,
                       ocols, oflows))
        return;
    purify_attempt(m, n, rows_in, cols_in, flows_in, costs_in, a, b, drop_rel, false, orows, ocols,
                   oflows);
}

}  // namespace otip
