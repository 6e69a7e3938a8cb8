// Graph nested dissection (Section 4.2 orders with nested dissection).  Multilevel
// bisection: heavy-edge matching coarsens the graph, a greedy-grown bisection of the
// coarsest graph is refined by boundary moves on the way back up, and the cut edges are
// turned into a vertex separator by a minimum vertex cover of the bipartite cut graph
// (König).  The two halves are ordered first (recursively), the separator last.  Small
// subgraphs, and subgraphs whose split does not lower the cost of factorising the subgraph
// against minimum degree, are ordered by minimum degree.  The cost counts flops plus the
// height of the elimination tree, since every pivot on the longest path is a sequential
// step on the device (order_cost).  Deterministic: every random order comes from a
// fixed-seed generator.
#include <algorithm>
#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace qdmf {

namespace {

struct Graph {
    int32_t n = 0;
    std::vector<int64_t> xa;
    std::vector<int32_t> ad;
    std::vector<int32_t> ew;  // edge weights
    std::vector<int32_t> vw;  // vertex weights
    int64_t total = 0;
};

struct Lcg {
    uint64_t s;
    explicit Lcg(uint64_t seed) : s(seed * 6364136223846793005ull + 1442695040888963407ull) {}
    uint32_t next() {
        s = s * 6364136223846793005ull + 1442695040888963407ull;
        return (uint32_t)(s >> 33);
    }
};

void shuffle(std::vector<int32_t>& v, Lcg& g) {
    for (size_t i = v.size(); i > 1; --i) std::swap(v[i - 1], v[g.next() % i]);
}

// Heavy-edge matching; returns false when the graph barely shrinks.
bool coarsen(const Graph& G, Graph& C, std::vector<int32_t>& cmap, Lcg& rng) {
    const int32_t n = G.n;
    std::vector<int32_t> match(n, -1), vis(n);
    for (int32_t i = 0; i < n; ++i) vis[i] = i;
    shuffle(vis, rng);
    cmap.assign(n, -1);
    int32_t nc = 0;
    for (int32_t u : vis) {
        if (match[u] >= 0) continue;
        int32_t best = u, bw = -1;
        for (int64_t e = G.xa[u]; e < G.xa[u + 1]; ++e) {
            const int32_t v = G.ad[e];
            if (match[v] < 0 && v != u && G.ew[e] > bw) {
                bw = G.ew[e];
                best = v;
            }
        }
        match[u] = best;
        match[best] = u;
        cmap[u] = cmap[best] = nc++;
    }
    if (nc > 0.9 * n) return false;
    C.n = nc;
    C.vw.assign(nc, 0);
    C.xa.assign(nc + 1, 0);
    C.ad.clear();
    C.ew.clear();
    C.total = G.total;
    std::vector<int32_t> mark(nc, -1), members;
    std::vector<std::vector<int32_t>> mem(nc);
    for (int32_t u = 0; u < n; ++u) mem[cmap[u]].push_back(u);
    for (int32_t c = 0; c < nc; ++c) {
        const int64_t start = (int64_t)C.ad.size();
        for (int32_t u : mem[c]) {
            C.vw[c] += G.vw[u];
            for (int64_t e = G.xa[u]; e < G.xa[u + 1]; ++e) {
                const int32_t d = cmap[G.ad[e]];
                if (d == c) continue;
                if (mark[d] >= start) {
                    C.ew[mark[d]] += G.ew[e];
                } else {
                    mark[d] = (int32_t)C.ad.size();
                    C.ad.push_back(d);
                    C.ew.push_back(G.ew[e]);
                }
            }
        }
        C.xa[c + 1] = (int64_t)C.ad.size();
    }
    return true;
}

int64_t cut_of(const Graph& G, const std::vector<int8_t>& part) {
    int64_t cut = 0;
    for (int32_t u = 0; u < G.n; ++u)
        for (int64_t e = G.xa[u]; e < G.xa[u + 1]; ++e)
            if (part[u] != part[G.ad[e]]) cut += G.ew[e];
    return cut / 2;
}

// Greedy boundary refinement: moves with positive gain (or zero gain that improves the
// balance) while both sides stay under the weight limit.
void refine(const Graph& G, std::vector<int8_t>& part, Lcg& rng, double bal) {
    const int64_t limit = (int64_t)(bal * G.total) + 1;
    int64_t w[2] = {0, 0};
    for (int32_t u = 0; u < G.n; ++u) w[part[u]] += G.vw[u];
    std::vector<int32_t> order(G.n);
    for (int32_t i = 0; i < G.n; ++i) order[i] = i;
    for (int pass = 0; pass < 6; ++pass) {
        shuffle(order, rng);
        int moves = 0;
        for (int32_t u : order) {
            int64_t in = 0, ex = 0;
            for (int64_t e = G.xa[u]; e < G.xa[u + 1]; ++e) (part[G.ad[e]] == part[u] ? in : ex) += G.ew[e];
            if (ex == 0) continue;
            const int8_t to = (int8_t)(1 - part[u]);
            if (w[to] + G.vw[u] > limit) continue;
            const int64_t gain = ex - in;
            if (gain > 0 || (gain == 0 && w[to] + G.vw[u] < w[part[u]])) {
                w[part[u]] -= G.vw[u];
                w[to] += G.vw[u];
                part[u] = to;
                ++moves;
            }
        }
        if (!moves) break;
    }
}

// Bisection of the coarsest graph: breadth-first growth from several seeds, refined; the
// best cut wins.
void initial_bisect(const Graph& G, std::vector<int8_t>& part, Lcg& rng, double bal) {
    int64_t best = -1;
    std::vector<int8_t> cand(G.n);
    for (int trial = 0; trial < 8; ++trial) {
        std::fill(cand.begin(), cand.end(), (int8_t)1);
        std::vector<int32_t> queue;
        queue.push_back((int32_t)(rng.next() % G.n));
        cand[queue[0]] = 0;
        int64_t w = G.vw[queue[0]];
        size_t head = 0;
        while (w < G.total / 2) {
            if (head == queue.size()) {  // disconnected: restart from an unvisited node
                int32_t v = -1;
                for (int32_t i = 0; i < G.n; ++i)
                    if (cand[i]) {
                        v = i;
                        break;
                    }
                if (v < 0) break;
                cand[v] = 0;
                w += G.vw[v];
                queue.push_back(v);
                continue;
            }
            const int32_t u = queue[head++];
            for (int64_t e = G.xa[u]; e < G.xa[u + 1] && w < G.total / 2; ++e) {
                const int32_t v = G.ad[e];
                if (cand[v]) {
                    cand[v] = 0;
                    w += G.vw[v];
                    queue.push_back(v);
                }
            }
        }
        refine(G, cand, rng, bal);
        const int64_t c = cut_of(G, cand);
        if (best < 0 || c < best) {
            best = c;
            part = cand;
        }
    }
}

// Multilevel bisection of G (unit weights on entry); no side above bal of the weight.
void bisect(const Graph& G0, std::vector<int8_t>& part, Lcg& rng, double bal) {
    std::vector<Graph> levels;
    std::vector<std::vector<int32_t>> maps;
    levels.push_back(G0);
    while (levels.back().n > 120) {
        Graph C;
        std::vector<int32_t> cmap;
        if (!coarsen(levels.back(), C, cmap, rng)) break;
        levels.push_back(std::move(C));
        maps.push_back(std::move(cmap));
    }
    initial_bisect(levels.back(), part, rng, bal);
    for (int l = (int)levels.size() - 2; l >= 0; --l) {
        std::vector<int8_t> fine(levels[l].n);
        for (int32_t u = 0; u < levels[l].n; ++u) fine[u] = part[maps[l][u]];
        part.swap(fine);
        refine(levels[l], part, rng, bal);
    }
}

// Minimum vertex cover of the bipartite graph of cut edges (König): maximum matching by
// augmenting paths, then the cover from the vertices reachable by alternating paths.
void vertex_separator(const Graph& G, const std::vector<int8_t>& part, std::vector<int8_t>& sep) {
    const int32_t n = G.n;
    sep.assign(n, 0);
    std::vector<int32_t> L, idx(n, -1);
    for (int32_t u = 0; u < n; ++u) {
        bool b = false;
        for (int64_t e = G.xa[u]; e < G.xa[u + 1] && !b; ++e) b = part[G.ad[e]] != part[u];
        if (b && part[u] == 0) {
            idx[u] = (int32_t)L.size();
            L.push_back(u);
        }
    }
    std::vector<int32_t> mate(n, -1);  // matched partner of any boundary vertex
    std::vector<int32_t> seen(n, -1);
    std::vector<std::pair<int32_t, int64_t>> stack;
    std::vector<int32_t> path;
    for (size_t li = 0; li < L.size(); ++li) {
        // iterative DFS for an augmenting path from L[li]
        stack.clear();
        path.clear();
        stack.push_back({L[li], G.xa[L[li]]});
        bool found = false;
        while (!stack.empty() && !found) {
            auto& top = stack.back();
            const int32_t u = top.first;
            bool pushed = false;
            while (top.second < G.xa[u + 1]) {
                const int32_t v = G.ad[top.second++];
                if (part[v] != 1 || seen[v] == (int32_t)li) continue;
                seen[v] = (int32_t)li;
                if (mate[v] < 0) {
                    // augment along the stack
                    int32_t cur = v;
                    for (int s = (int)stack.size() - 1; s >= 0; --s) {
                        const int32_t a = stack[s].first;
                        const int32_t prev = mate[a];
                        mate[a] = cur;
                        mate[cur] = a;
                        cur = prev;
                    }
                    found = true;
                    break;
                }
                stack.push_back({mate[v], G.xa[mate[v]]});
                pushed = true;
                break;
            }
            if (!found && !pushed) stack.pop_back();
        }
    }
    // Z: reachable from unmatched left vertices by alternating paths
    std::vector<int8_t> z(n, 0);
    std::vector<int32_t> q;
    for (int32_t u : L)
        if (mate[u] < 0) {
            z[u] = 1;
            q.push_back(u);
        }
    for (size_t h = 0; h < q.size(); ++h) {
        const int32_t u = q[h];
        if (part[u] == 0) {
            for (int64_t e = G.xa[u]; e < G.xa[u + 1]; ++e) {
                const int32_t v = G.ad[e];
                if (part[v] == 1 && !z[v] && mate[u] != v) {
                    z[v] = 1;
                    q.push_back(v);
                }
            }
        } else if (mate[u] >= 0 && !z[mate[u]]) {
            z[mate[u]] = 1;
            q.push_back(mate[u]);
        }
    }
    for (int32_t u : L)
        if (!z[u]) sep[u] = 1;
    for (int32_t u = 0; u < n; ++u)
        if (part[u] == 1 && z[u] && mate[u] >= 0) sep[u] = 1;
}

struct Nd {
    const std::vector<int64_t>* xadj;
    const std::vector<int32_t>* adj;
    std::vector<int32_t> local;
    Lcg rng{12345};
    int32_t leaf = 200;
};

void induced(Nd& S, const std::vector<int32_t>& nodes, Graph& G) {
    const auto& xadj = *S.xadj;
    const auto& adj = *S.adj;
    const int32_t k = (int32_t)nodes.size();
    for (int32_t i = 0; i < k; ++i) S.local[nodes[i]] = i;
    G.n = k;
    G.xa.assign(k + 1, 0);
    G.ad.clear();
    for (int32_t i = 0; i < k; ++i) {
        for (int64_t e = xadj[nodes[i]]; e < xadj[nodes[i] + 1]; ++e)
            if (S.local[adj[e]] >= 0) G.ad.push_back(S.local[adj[e]]);
        G.xa[i + 1] = (int64_t)G.ad.size();
    }
    for (int32_t v : nodes) S.local[v] = -1;
    G.ew.assign(G.ad.size(), 1);
    G.vw.assign(k, 1);
    G.total = k;
}

void amd_of(const std::vector<int32_t>& nodes, const Graph& G, std::vector<int32_t>& out) {
    std::vector<int32_t> ord;
    amd_order(G.n, G.xa, G.ad, ord);
    out.clear();
    for (int32_t i : ord) out.push_back(nodes[i]);
}

// Orders nodes into out.  A split is kept only when the subgraph's factorisation is cheaper
// with it than with minimum degree on the whole subgraph.
void dissect(Nd& S, const std::vector<int32_t>& nodes, std::vector<int32_t>& out) {
    Graph G;
    induced(S, nodes, G);
    // connected components, each on its own
    std::vector<int32_t> comp(G.n, -1);
    int32_t nc = 0;
    std::vector<int32_t> q;
    for (int32_t s = 0; s < G.n; ++s) {
        if (comp[s] >= 0) continue;
        q.assign(1, s);
        comp[s] = nc;
        for (size_t h = 0; h < q.size(); ++h)
            for (int64_t e = G.xa[q[h]]; e < G.xa[q[h] + 1]; ++e)
                if (comp[G.ad[e]] < 0) {
                    comp[G.ad[e]] = nc;
                    q.push_back(G.ad[e]);
                }
        ++nc;
    }
    if (nc > 1) {
        std::vector<std::vector<int32_t>> parts(nc);
        for (int32_t i = 0; i < G.n; ++i) parts[comp[i]].push_back(nodes[i]);
        out.clear();
        std::vector<int32_t> sub;
        for (auto& p : parts) {
            dissect(S, p, sub);
            out.insert(out.end(), sub.begin(), sub.end());
        }
        return;
    }
    if (G.n <= S.leaf) {
        amd_of(nodes, G, out);
        return;
    }
    // vertex separators from a balanced and a looser bisection; the smaller ratio
    // |S| / min(|A|, |B|) wins (a chain of weakly linked blocks is cut at a link)
    std::vector<int32_t> A, B, Sv;
    double best = -1.0;
    for (double bal : {0.53, 0.7}) {
        std::vector<int8_t> part, sep;
        bisect(G, part, S.rng, bal);
        vertex_separator(G, part, sep);
        std::vector<int32_t> a, b, sv;
        for (int32_t i = 0; i < G.n; ++i) (sep[i] ? sv : (part[i] ? b : a)).push_back(nodes[i]);
        const double side = (double)std::min(a.size(), b.size());
        const double ratio = side > 0 ? (double)sv.size() / side : 1e30;
        if (best < 0 || ratio < best) {
            best = ratio;
            A.swap(a);
            B.swap(b);
            Sv.swap(sv);
        }
    }
    if (A.empty() || B.empty() || (int64_t)Sv.size() * 3 > G.n) {
        amd_of(nodes, G, out);
        return;
    }
    std::vector<int32_t> oa, ob;
    dissect(S, A, oa);
    dissect(S, B, ob);
    out = oa;
    out.insert(out.end(), ob.begin(), ob.end());
    out.insert(out.end(), Sv.begin(), Sv.end());
    // compare with minimum degree on this subgraph (local numbering)
    std::vector<int32_t> amd_local, nd_local(G.n);
    amd_order(G.n, G.xa, G.ad, amd_local);
    for (int32_t i = 0; i < G.n; ++i) S.local[nodes[i]] = i;
    for (int32_t i = 0; i < G.n; ++i) nd_local[i] = S.local[out[i]];
    for (int32_t v : nodes) S.local[v] = -1;
    if (order_cost(G.n, G.xa, G.ad, amd_local) <= order_cost(G.n, G.xa, G.ad, nd_local)) {
        out.clear();
        for (int32_t i : amd_local) out.push_back(nodes[i]);
    }
}

}  // namespace

void nd_order(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
              std::vector<int32_t>& order) {
    Nd S;
    S.xadj = &xadj;
    S.adj = &adj;
    S.local.assign(N, -1);
    std::vector<int32_t> all(N);
    for (int32_t i = 0; i < N; ++i) all[i] = i;
    dissect(S, all, order);
}

}  // namespace qdmf
