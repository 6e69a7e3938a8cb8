// Symbolic analysis on the host, run once per pattern (Section 4.2): K pattern, ordering,
// elimination tree (Section 4.3), postorder, column structures, supernodes and relaxed
// amalgamation (Section 4.1), child->parent index maps, the entry->front map, the
// normal-equation product lists, levels of the supernodal tree and the launch plan.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>
#include <atomic>
#include <thread>

#include "../../include/qdmf.h"
#include "plan.hpp"

namespace qdmf {

namespace {

int check_csc(int32_t m, int32_t n, const int64_t* cp, const int32_t* ri, std::string& msg) {
    if (m < 0 || n < 0 || !cp || (!ri && n > 0 && cp[n] > 0)) {
        msg = "null or negative argument";
        return QDMF_ERR_INVALID_ARG;
    }
    if (cp[0] != 0) {
        msg = "colptr[0] != 0";
        return QDMF_ERR_INVALID_ARG;
    }
    for (int32_t j = 0; j < n; ++j) {
        if (cp[j + 1] < cp[j]) {
            msg = "colptr not monotone";
            return QDMF_ERR_INVALID_ARG;
        }
        for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
            if (ri[e] < 0 || ri[e] >= m) {
                msg = "row index out of range";
                return QDMF_ERR_INVALID_ARG;
            }
            if (e > cp[j] && ri[e] <= ri[e - 1]) {
                msg = "row indices not strictly increasing within a column";
                return QDMF_ERR_INVALID_ARG;
            }
        }
    }
    if (cp[n] > INT32_MAX) {
        msg = "more than 2^31-1 nonzeros in A";
        return QDMF_ERR_INDEX_OVERFLOW;
    }
    return 0;
}

// Full adjacency of K (no diagonal), original numbering.  AS: x_j -- y_i where A_ij != 0, and
// for a quadratic program x_j -- x_k where Q_jk != 0 (j != k); each list ascending.
void k_adjacency(const Plan& P, std::vector<int64_t>& xadj, std::vector<int32_t>& adj) {
    const int32_t N = P.N, n = P.n, m = P.m;
    xadj.assign(N + 1, 0);
    if (P.mode == QDMF_AS) {
        auto qoff = [&](int32_t j) {
            if (!P.has_q) return (int64_t)0;
            return P.qfcp[j + 1] - P.qfcp[j] - (P.qdiag[j] >= 0 ? 1 : 0);
        };
        for (int32_t j = 0; j < n; ++j) xadj[j + 1] = qoff(j) + P.acp[j + 1] - P.acp[j];
        for (int32_t i = 0; i < m; ++i) xadj[n + i + 1] = P.arp[i + 1] - P.arp[i];
        for (int32_t v = 0; v < N; ++v) xadj[v + 1] += xadj[v];
        adj.resize(xadj[N]);
        for (int32_t j = 0; j < n; ++j) {
            int64_t w = xadj[j];
            if (P.has_q)
                for (int64_t e = P.qfcp[j]; e < P.qfcp[j + 1]; ++e)
                    if (P.qfri[e] != j) adj[w++] = P.qfri[e];
            for (int64_t e = P.acp[j]; e < P.acp[j + 1]; ++e) adj[w++] = n + P.ari[e];
        }
        for (int32_t i = 0; i < m; ++i)
            for (int64_t q = P.arp[i]; q < P.arp[i + 1]; ++q)
                adj[xadj[n + i] + (q - P.arp[i])] = P.acol[P.are[q]];
    } else {
        std::vector<int32_t> mark(m, -1);
        std::vector<int32_t> tmp;
        std::vector<std::vector<int32_t>> rowsv(m);
        for (int32_t i = 0; i < m; ++i) {
            tmp.clear();
            mark[i] = i;
            for (int64_t q = P.arp[i]; q < P.arp[i + 1]; ++q) {
                int32_t j = P.acol[P.are[q]];
                for (int64_t e = P.acp[j]; e < P.acp[j + 1]; ++e) {
                    int32_t k = P.ari[e];
                    if (mark[k] != i) {
                        mark[k] = i;
                        tmp.push_back(k);
                    }
                }
            }
            std::sort(tmp.begin(), tmp.end());
            rowsv[i] = tmp;
            xadj[i + 1] = xadj[i] + (int64_t)tmp.size();
        }
        adj.resize(xadj[N]);
        for (int32_t i = 0; i < m; ++i) std::copy(rowsv[i].begin(), rowsv[i].end(), adj.begin() + xadj[i]);
    }
}

// Liu's elimination tree algorithm with path compression, order given by iorder (old->new).
void etree(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
           const std::vector<int32_t>& order, const std::vector<int32_t>& iorder,
           std::vector<int32_t>& parent) {
    parent.assign(N, -1);
    std::vector<int32_t> anc(N, -1);
    for (int32_t j = 0; j < N; ++j) {
        int32_t old = order[j];
        for (int64_t e = xadj[old]; e < xadj[old + 1]; ++e) {
            int32_t i = iorder[adj[e]];
            if (i >= j) continue;
            while (anc[i] != -1 && anc[i] != j) {
                int32_t t = anc[i];
                anc[i] = j;
                i = t;
            }
            if (anc[i] == -1) {
                anc[i] = j;
                parent[i] = j;
            }
        }
    }
}

}  // namespace

// Column counts of L (entries below the diagonal) and the elimination tree of an ordering,
// from the row subtrees.
static void order_counts(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
                         const std::vector<int32_t>& order, std::vector<int64_t>& cnt,
                         std::vector<int32_t>& parent) {
    std::vector<int32_t> iorder(N), mark(N, -1);
    for (int32_t k = 0; k < N; ++k) iorder[order[k]] = k;
    etree(N, xadj, adj, order, iorder, parent);
    cnt.assign(N, 0);
    for (int32_t i = 0; i < N; ++i) {
        const int32_t old = order[i];
        mark[i] = i;
        for (int64_t e = xadj[old]; e < xadj[old + 1]; ++e) {
            int32_t j = iorder[adj[e]];
            while (j >= 0 && j < i && mark[j] != i) {
                mark[j] = i;
                ++cnt[j];
                j = parent[j];
            }
        }
    }
}

// Factorisation flops sum_j c_j (c_j + 3) of an ordering (c_j = entries of column j of L
// below the diagonal).
double order_flops(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
                   const std::vector<int32_t>& order) {
    std::vector<int64_t> cnt;
    std::vector<int32_t> parent;
    order_counts(N, xadj, adj, order, cnt, parent);
    double fl = 0;
    for (int32_t j = 0; j < N; ++j) fl += (double)cnt[j] * (cnt[j] + 3);
    return fl;
}

// Flops plus the height of the elimination tree weighted as 2e6 flops per level: on the
// device every pivot on the longest path is a sequential step of roughly a microsecond,
// during which the matrix units could have done that many flops.
double order_cost(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
                  const std::vector<int32_t>& order) {
    std::vector<int64_t> cnt;
    std::vector<int32_t> parent;
    order_counts(N, xadj, adj, order, cnt, parent);
    double fl = 0;
    std::vector<int32_t> h(N, 1);
    int32_t height = 0;
    for (int32_t j = 0; j < N; ++j) {
        fl += (double)cnt[j] * (cnt[j] + 3);
        height = std::max(height, h[j]);
        if (parent[j] >= 0) h[parent[j]] = std::max(h[parent[j]], h[j] + 1);
    }
    return fl + 2e6 * height;
}

namespace {

// Fill-reducing order of one subgraph (nodes listed in nodes) by the handle's method.
void order_one(int32_t ordering, const std::vector<int32_t>& nodes, const std::vector<int64_t>& xadj,
               const std::vector<int32_t>& adj, std::vector<int32_t>& local, std::vector<int32_t>& out) {
    const int32_t k = (int32_t)nodes.size();
    for (int32_t i = 0; i < k; ++i) local[nodes[i]] = i;
    std::vector<int64_t> sx(k + 1, 0);
    std::vector<int32_t> sa;
    for (int32_t i = 0; i < k; ++i) {
        for (int64_t e = xadj[nodes[i]]; e < xadj[nodes[i] + 1]; ++e)
            if (local[adj[e]] >= 0) sa.push_back(local[adj[e]]);
        sx[i + 1] = (int64_t)sa.size();
    }
    for (int32_t v : nodes) local[v] = -1;
    std::vector<int32_t> ord;
    if (ordering == QDMF_ORDER_ND) {
        nd_order(k, sx, sa, ord);
    } else {
        amd_order(k, sx, sa, ord);
        if (ordering == QDMF_ORDER_AUTO) {
            std::vector<int32_t> nd;
            nd_order(k, sx, sa, nd);
            if (order_cost(k, sx, sa, nd) < order_cost(k, sx, sa, ord)) ord.swap(nd);
        }
    }
    out.resize(k);
    for (int32_t i = 0; i < k; ++i) out[i] = nodes[ord[i]];
}

// Batch: the systems are the diagonal blocks, ordered independently by a pool of threads;
// the order is the systems' orders concatenated (deterministic).
void order_systems(int32_t N, int32_t m, int32_t n, int32_t mode, const AnalyseOptions& opt,
                   const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj, std::vector<int32_t>& order) {
    const int32_t ns = opt.nsys;
    std::vector<std::vector<int32_t>> nodes(ns), outs(ns);
    for (int32_t q = 0; q < ns; ++q) {
        if (mode == QDMF_AS)
            for (int64_t j = opt.col_off[q]; j < opt.col_off[q + 1]; ++j) nodes[q].push_back((int32_t)j);
        for (int64_t i = opt.row_off[q]; i < opt.row_off[q + 1]; ++i)
            nodes[q].push_back((int32_t)(mode == QDMF_AS ? n + i : i));
    }
    (void)m;
    std::atomic<int32_t> next(0);
    const int32_t nt = std::max(1, std::min<int32_t>(ns, (int32_t)std::thread::hardware_concurrency()));
    std::vector<std::thread> pool;
    for (int32_t t = 0; t < nt; ++t)
        pool.emplace_back([&]() {
            std::vector<int32_t> local(N, -1);
            for (int32_t q; (q = next++) < ns;) order_one(opt.ordering, nodes[q], xadj, adj, local, outs[q]);
        });
    for (auto& th : pool) th.join();
    order.clear();
    order.reserve(N);
    for (int32_t q = 0; q < ns; ++q) order.insert(order.end(), outs[q].begin(), outs[q].end());
}

void postorder(int32_t N, const std::vector<int32_t>& parent, std::vector<int32_t>& post) {
    std::vector<int32_t> head(N, -1), nxt(N, -1), stack;
    for (int32_t j = N - 1; j >= 0; --j)
        if (parent[j] >= 0) {
            nxt[j] = head[parent[j]];
            head[parent[j]] = j;
        }
    post.clear();
    post.reserve(N);
    for (int32_t r = 0; r < N; ++r) {
        if (parent[r] >= 0) continue;
        stack.push_back(r);
        while (!stack.empty()) {
            int32_t v = stack.back();
            int32_t c = head[v];
            if (c >= 0) {
                head[v] = nxt[c];
                stack.push_back(c);
            } else {
                post.push_back(v);
                stack.pop_back();
            }
        }
    }
}

int32_t find_pos(const int32_t* rows, int32_t c0, int32_t p, int32_t f, int32_t r) {
    if (r >= c0 && r < c0 + p) return r - c0;
    const int32_t* b = rows + p;
    const int32_t* e = rows + f;
    const int32_t* it = std::lower_bound(b, e, r);
    if (it == e || *it != r) return -1;
    return (int32_t)(it - rows);
}

}  // namespace

int64_t ne_pattern_count(int32_t m, int32_t n, const int64_t* colptr, const int32_t* rowidx, int64_t limit) {
    // rows of A as lists of columns
    std::vector<int64_t> rp(m + 1, 0);
    for (int64_t e = 0; e < colptr[n]; ++e) rp[rowidx[e] + 1]++;
    for (int32_t i = 0; i < m; ++i) rp[i + 1] += rp[i];
    std::vector<int32_t> rc(colptr[n]);
    {
        std::vector<int64_t> fill(rp.begin(), rp.end() - 1);
        for (int32_t j = 0; j < n; ++j)
            for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) rc[fill[rowidx[e]]++] = j;
    }
    std::vector<int32_t> mark(m, -1);
    int64_t count = 0;
    for (int32_t i = 0; i < m; ++i) {  // row i of the lower triangle: rows k <= i sharing a column
        for (int64_t q = rp[i]; q < rp[i + 1]; ++q) {
            const int32_t j = rc[q];
            for (int64_t e = colptr[j]; e < colptr[j + 1] && rowidx[e] <= i; ++e) {
                const int32_t k = rowidx[e];
                if (mark[k] != i) {
                    mark[k] = i;
                    if (++count > limit) return count;
                }
            }
        }
        if (mark[i] != i) {  // the diagonal (delta > 0) even for an empty row
            mark[i] = i;
            if (++count > limit) return count;
        }
    }
    return count;
}

// pivot columns of one window of the factorisation kernels (Section 4.4's block of nb columns)
constexpr int64_t AMALG_WINDOW = 64;
// smallest front that joins a level's multi-workgroup solve launches
constexpr int32_t SPLIT_JOIN_FRONT = 128;

// Q's lower triangle: rows >= the column, strictly increasing, inside [0, n); the full
// symmetric pattern with the source of each value, and the diagonal positions.
static int set_hessian_pattern(int32_t n, const int64_t* qcp, const int32_t* qri, Plan& P, std::string& msg) {
    if (qcp[0] != 0) {
        msg = "Q: colptr[0] must be 0";
        return QDMF_ERR_INVALID_ARG;
    }
    for (int32_t j = 0; j < n; ++j) {
        if (qcp[j + 1] < qcp[j]) {
            msg = "Q: colptr not nondecreasing";
            return QDMF_ERR_INVALID_ARG;
        }
        for (int64_t e = qcp[j]; e < qcp[j + 1]; ++e) {
            if (qri[e] < j || qri[e] >= n) {
                msg = "Q: entries must lie in the lower triangle (row >= column, row < n)";
                return QDMF_ERR_INVALID_ARG;
            }
            if (e > qcp[j] && qri[e] <= qri[e - 1]) {
                msg = "Q: row indices not strictly increasing within a column";
                return QDMF_ERR_INVALID_ARG;
            }
        }
    }
    if (qcp[n] > INT32_MAX) {
        msg = "more than 2^31-1 nonzeros in Q";
        return QDMF_ERR_INDEX_OVERFLOW;
    }
    const int64_t qnnz = qcp[n];
    P.has_q = true;
    P.qcp.assign(qcp, qcp + n + 1);
    P.qri.assign(qri, qri + qnnz);
    P.qdiag.assign(n, -1);
    P.qfcp.assign(n + 1, 0);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t e = qcp[j]; e < qcp[j + 1]; ++e) {
            P.qfcp[j + 1]++;
            if (qri[e] != j) P.qfcp[qri[e] + 1]++;
            else P.qdiag[j] = e;
        }
    for (int32_t j = 0; j < n; ++j) P.qfcp[j + 1] += P.qfcp[j];
    P.qfri.resize(P.qfcp[n]);
    P.qfsrc.resize(P.qfcp[n]);
    std::vector<int64_t> fl(P.qfcp.begin(), P.qfcp.end() - 1);
    // column k of the full pattern: first the upper entries (rows j < k, from the lower
    // triangle's columns j in ascending order), then column k of the lower triangle
    for (int32_t j = 0; j < n; ++j)
        for (int64_t e = qcp[j]; e < qcp[j + 1]; ++e) {
            const int32_t k = qri[e];
            if (k != j) {
                P.qfri[fl[k]] = j;
                P.qfsrc[fl[k]++] = e;
            }
        }
    for (int32_t j = 0; j < n; ++j)
        for (int64_t e = qcp[j]; e < qcp[j + 1]; ++e) {
            P.qfri[fl[j]] = qri[e];
            P.qfsrc[fl[j]++] = e;
        }
    return 0;
}

int build_plan(int32_t m, int32_t n, const int64_t* colptr, const int32_t* rowidx, int32_t mode,
               const AnalyseOptions& opt, Plan& P, std::string& msg) {
    if (mode != QDMF_NE && mode != QDMF_AS) {
        msg = "mode must be QDMF_NE or QDMF_AS";
        return QDMF_ERR_INVALID_ARG;
    }
    int rc = check_csc(m, n, colptr, rowidx, msg);
    if (rc) return rc;
    if (mode == QDMF_AS && (int64_t)n + m > INT32_MAX) {
        msg = "n + m exceeds 2^31-1";
        return QDMF_ERR_INDEX_OVERFLOW;
    }
    P = Plan();
    P.m = m;
    P.n = n;
    P.mode = mode;
    P.N = mode == QDMF_AS ? n + m : m;
    const int32_t N = P.N;
    const int64_t annz = colptr[n];
    P.acp.assign(colptr, colptr + n + 1);
    P.long_col.clear();
    P.long_of.assign(n, -1);
    if (mode == 1)
        for (int32_t c = 0; c < n; ++c)
            if (colptr[c + 1] - colptr[c] > LONG_COL) {
                P.long_of[c] = (int32_t)P.long_col.size();
                P.long_col.push_back(c);
            }
    P.ari.assign(rowidx, rowidx + annz);
    P.acol.resize(annz);
    for (int32_t j = 0; j < n; ++j)
        for (int64_t e = colptr[j]; e < colptr[j + 1]; ++e) P.acol[e] = j;
    P.arp.assign(m + 1, 0);
    for (int64_t e = 0; e < annz; ++e) P.arp[rowidx[e] + 1]++;
    for (int32_t i = 0; i < m; ++i) P.arp[i + 1] += P.arp[i];
    P.are.resize(annz);
    {
        std::vector<int64_t> fill(P.arp.begin(), P.arp.end() - 1);
        for (int64_t e = 0; e < annz; ++e) P.are[fill[rowidx[e]]++] = (int32_t)e;
    }
    if (opt.q_colptr) {
        if (mode != QDMF_AS || opt.nsys > 1) {
            msg = "a quadratic program needs the augmented system of one system";
            return QDMF_ERR_UNSUPPORTED;
        }
        if (n > 0 && !opt.q_rowidx && opt.q_colptr[n] > 0) {
            msg = "Q: missing row indices";
            return QDMF_ERR_INVALID_ARG;
        }
        rc = set_hessian_pattern(n, opt.q_colptr, opt.q_rowidx, P, msg);
        if (rc) return rc;
    }

    std::vector<int64_t> xadj;
    std::vector<int32_t> adj;
    k_adjacency(P, xadj, adj);

    // ----- ordering
    std::vector<int32_t> order;
    if (opt.ordering == QDMF_ORDER_USER) {
        if (!opt.user_perm) {
            msg = "user ordering requested without a permutation";
            return QDMF_ERR_INVALID_ARG;
        }
        order.assign(opt.user_perm, opt.user_perm + N);
    } else if (opt.ordering == QDMF_ORDER_GRID_ND) {
        if ((int64_t)opt.grid[0] * opt.grid[1] * opt.grid[2] != m) {
            msg = "grid dims do not multiply to m";
            return QDMF_ERR_INVALID_ARG;
        }
        grid_nd_order(P, opt.grid, xadj, adj, order);
    } else if (opt.nsys > 1) {  // a batch: each system ordered on its own, in parallel
        order_systems(N, m, n, mode, opt, xadj, adj, order);
    } else if (opt.ordering == QDMF_ORDER_ND) {
        nd_order(N, xadj, adj, order);
    } else if (opt.ordering == QDMF_ORDER_AUTO) {  // the cheaper of the two (order_cost)
        std::vector<int32_t> nd;
        amd_order(N, xadj, adj, order);
        nd_order(N, xadj, adj, nd);
        if (order_cost(N, xadj, adj, nd) < order_cost(N, xadj, adj, order)) order.swap(nd);
    } else {
        amd_order(N, xadj, adj, order);
    }
    std::vector<int32_t> iorder(N, -1);
    if ((int32_t)order.size() != N) {
        msg = "ordering has the wrong length";
        return QDMF_ERR_INVALID_ARG;
    }
    for (int32_t k = 0; k < N; ++k) {
        if (order[k] < 0 || order[k] >= N || iorder[order[k]] >= 0) {
            msg = "ordering is not a permutation";
            return QDMF_ERR_INVALID_ARG;
        }
        iorder[order[k]] = k;
    }

    // ----- elimination tree, postorder (children ascending)
    std::vector<int32_t> par0, post;
    etree(N, xadj, adj, order, iorder, par0);
    postorder(N, par0, post);
    P.perm.resize(N);
    P.iperm.resize(N);
    for (int32_t k = 0; k < N; ++k) P.perm[k] = order[post[k]];
    for (int32_t k = 0; k < N; ++k) P.iperm[P.perm[k]] = k;
    std::vector<int32_t> ipost(N), parent(N, -1);
    for (int32_t k = 0; k < N; ++k) ipost[post[k]] = k;
    for (int32_t k = 0; k < N; ++k) parent[k] = par0[post[k]] >= 0 ? ipost[par0[post[k]]] : -1;
    std::vector<int32_t>().swap(par0);
    std::vector<int32_t>().swap(post);

    // ----- column structures (freed as soon as they are consumed), fundamental supernodes
    std::vector<int32_t> nkids(N, 0);
    for (int32_t j = 0; j < N; ++j)
        if (parent[j] >= 0) nkids[parent[j]]++;
    std::vector<int32_t> kid_ptr(N + 1, 0), kid(N);
    for (int32_t j = 0; j < N; ++j)
        if (parent[j] >= 0) kid_ptr[parent[j] + 1]++;
    for (int32_t j = 0; j < N; ++j) kid_ptr[j + 1] += kid_ptr[j];
    {
        std::vector<int32_t> fl(kid_ptr.begin(), kid_ptr.end() - 1);
        for (int32_t j = 0; j < N; ++j)
            if (parent[j] >= 0) kid[fl[parent[j]]++] = j;
    }
    std::vector<std::vector<int32_t>> cs(N);
    std::vector<int64_t> cc(N, 0);
    std::vector<int32_t> mark(N, -1);
    std::vector<char> sn_start(N, 0);
    P.nnz_l = 0;
    P.flops_fact = 0;
    for (int32_t j = 0; j < N; ++j) {
        std::vector<int32_t> S;
        int32_t old = P.perm[j];
        for (int64_t e = xadj[old]; e < xadj[old + 1]; ++e) {
            int32_t i = P.iperm[adj[e]];
            if (i > j && mark[i] != j) {
                mark[i] = j;
                S.push_back(i);
            }
        }
        for (int32_t q = kid_ptr[j]; q < kid_ptr[j + 1]; ++q)
            for (int32_t i : cs[kid[q]])
                if (i != j && mark[i] != j) {
                    mark[i] = j;
                    S.push_back(i);
                }
        std::sort(S.begin(), S.end());
        cc[j] = (int64_t)S.size() + 1;
        P.nnz_l += cc[j];
        P.flops_fact += (double)S.size() * ((double)S.size() + 3.0);
        bool join = j > 0 && parent[j - 1] == j && nkids[j] == 1 && cc[j - 1] == cc[j] + 1;
        sn_start[j] = !join;
        if (join) std::vector<int32_t>().swap(cs[j - 1]);  // interior column: not needed
        cs[j] = std::move(S);
    }
    P.flops_solve = 4.0 * (double)(P.nnz_l - N) + N;

    // fundamental supernodes: start, ncols, struct of last column (kept in cs)
    std::vector<int32_t> s_start, s_p;
    for (int32_t j = 0; j < N; ++j)
        if (sn_start[j]) s_start.push_back(j);
    int32_t ns0 = (int32_t)s_start.size();
    s_p.resize(ns0);
    for (int32_t s = 0; s < ns0; ++s) s_p[s] = (s + 1 < ns0 ? s_start[s + 1] : N) - s_start[s];
    std::vector<int32_t> col2sn(N);
    for (int32_t s = 0; s < ns0; ++s)
        for (int32_t c = s_start[s]; c < s_start[s] + s_p[s]; ++c) col2sn[c] = s;
    std::vector<int32_t> s_par(ns0, -1);
    for (int32_t s = 0; s < ns0; ++s) {
        int32_t last = s_start[s] + s_p[s] - 1;
        s_par[s] = parent[last] >= 0 ? col2sn[parent[last]] : -1;
    }

    // ----- relaxed amalgamation: merge the child whose columns immediately precede the
    // parent's, when it adds few explicit zeros (merged supernodes stay contiguous)
    std::vector<int32_t> alive(ns0, 1), s_nk(ns0, 0);
    std::vector<int64_t> s_zero(ns0, 0);
    std::vector<int32_t> s_last(ns0);  // index of the supernode holding the struct (the last fundamental)
    for (int32_t s = 0; s < ns0; ++s) {
        s_last[s] = s;
        if (s_par[s] >= 0) s_nk[s_par[s]]++;
    }
    auto fsize = [&](int32_t s) { return (int64_t)s_p[s] + (int64_t)cs[s_start[s] + s_p[s] - 1].size(); };
    std::vector<int64_t> s_f(ns0);
    for (int32_t s = 0; s < ns0; ++s) s_f[s] = fsize(s);
    std::vector<int32_t> merged_into(ns0, -1);
    // children of the alive supernodes and the height of each finished one (0 for a leaf): the
    // tree levels the launch plan will follow
    std::vector<std::vector<int32_t>> s_kids(ns0);
    for (int32_t s = 0; s < ns0; ++s)
        if (s_par[s] >= 0) s_kids[s_par[s]].push_back(s);
    std::vector<int32_t> s_h(ns0, 0);
    if (opt.amalgamate) {
        for (int32_t s = 0; s < ns0; ++s) {
            for (;;) {
                // adjacent child: the alive supernode ending at s_start[s]-1 whose parent is s
                if (s_start[s] == 0) break;
                int32_t c = col2sn[s_start[s] - 1];
                while (merged_into[c] >= 0) c = merged_into[c];
                if (!alive[c] || c == s) break;
                {
                    int32_t pc0 = s_par[c];
                    while (pc0 >= 0 && merged_into[pc0] >= 0) pc0 = merged_into[pc0];
                    if (pc0 != s) break;
                }
                int64_t delta = s_p[c] + s_f[s] - s_f[c];
                int64_t pc = s_p[c], pm = s_p[c] + s_p[s];
                int64_t fm = s_f[s] + s_p[c];
                int64_t ent = pm * fm - pm * (pm - 1) / 2;
                int64_t zeros = s_zero[c] + s_zero[s] + pc * delta;
                // (the third rule: large nearly dense fronts, whose separate square storage
                // and pivot windows would cost more than the few zeros; the fourth: a merged
                // supernode that still fits one pivot window, which saves the child's
                // contribution-block copy and, on chains of such supernodes, tree levels,
                // without lengthening the sequence of pivot steps of the level it lands on)
                bool ok = (s_nk[s] == 1 && delta <= 8) || (pc < 16 && (double)zeros <= 0.05 * (double)ent) ||
                          (fm >= 512 && (double)zeros <= 0.01 * (double)ent);
                if (!ok && pm <= AMALG_WINDOW && (double)zeros <= 0.05 * (double)ent) {
                    // the fourth rule only on chains: every other child of s is a leaf, so c
                    // alone sets s's level and the merge removes a level of the subtree
                    ok = true;
                    for (int32_t k : s_kids[s])
                        if (k != c && s_h[k] > 0) ok = false;
                }
                if (!ok) break;
                // merge c into s
                alive[c] = 0;
                merged_into[c] = s;
                s_start[s] = s_start[c];
                s_p[s] = (int32_t)pm;
                s_f[s] = fm;
                s_zero[s] = zeros;
                s_nk[s] += s_nk[c] - 1;
                auto& ks = s_kids[s];
                ks.erase(std::find(ks.begin(), ks.end(), c));
                ks.insert(ks.end(), s_kids[c].begin(), s_kids[c].end());
                std::vector<int32_t>().swap(s_kids[c]);
            }
            for (int32_t k : s_kids[s]) s_h[s] = std::max(s_h[s], s_h[k] + 1);
        }
    }
    // resolve parents through merges, renumber alive supernodes (ascending start = postorder)
    auto root_of = [&](int32_t s) {
        while (s >= 0 && merged_into[s] >= 0) s = merged_into[s];
        return s;
    };
    std::vector<int32_t> newid(ns0, -1);
    int32_t ns = 0;
    for (int32_t s = 0; s < ns0; ++s)
        if (alive[s]) newid[s] = ns++;
    P.ns = ns;
    P.sn_ptr.resize(ns + 1);
    P.sn_parent.assign(ns, -1);
    P.sn_f.resize(ns);
    P.sn_p.resize(ns);
    std::vector<int32_t> s_old(ns);
    for (int32_t s = 0; s < ns0; ++s) {
        if (!alive[s]) continue;
        int32_t t = newid[s];
        s_old[t] = s;
        P.sn_ptr[t] = s_start[s];
        P.sn_p[t] = s_p[s];
        int64_t f = s_f[s];
        if (f > INT32_MAX) {
            msg = "front order overflows int32";
            return QDMF_ERR_INDEX_OVERFLOW;
        }
        P.sn_f[t] = (int32_t)f;
        int32_t ps = root_of(s_par[s]);
        P.sn_parent[t] = ps >= 0 ? newid[ps] : -1;
    }
    P.sn_ptr[ns] = N;
    // row lists: pivot columns, then the structure of the last column
    P.sn_rowptr.assign(ns + 1, 0);
    for (int32_t t = 0; t < ns; ++t) P.sn_rowptr[t + 1] = P.sn_rowptr[t] + P.sn_f[t];
    P.rows.resize(P.sn_rowptr[ns]);
    for (int32_t t = 0; t < ns; ++t) {
        int32_t s = s_old[t];
        int64_t w = P.sn_rowptr[t];
        for (int32_t c = P.sn_ptr[t]; c < P.sn_ptr[t] + P.sn_p[t]; ++c) P.rows[w++] = c;
        const auto& st = cs[s_start[s] + s_p[s] - 1];  // unchanged by merging into s
        for (int32_t r : st) P.rows[w++] = r;
    }
    std::vector<std::vector<int32_t>>().swap(cs);
    P.max_front = 0;
    for (int32_t t = 0; t < ns; ++t) P.max_front = std::max(P.max_front, P.sn_f[t]);

    // children (ascending), levels
    P.ch_ptr.assign(ns + 1, 0);
    for (int32_t t = 0; t < ns; ++t)
        if (P.sn_parent[t] >= 0) P.ch_ptr[P.sn_parent[t] + 1]++;
    for (int32_t t = 0; t < ns; ++t) P.ch_ptr[t + 1] += P.ch_ptr[t];
    P.ch.resize(P.ch_ptr[ns]);
    {
        std::vector<int32_t> fl(P.ch_ptr.begin(), P.ch_ptr.end() - 1);
        for (int32_t t = 0; t < ns; ++t)
            if (P.sn_parent[t] >= 0) P.ch[fl[P.sn_parent[t]]++] = t;
    }
    P.sn_level.assign(ns, 0);
    P.nlevels = ns ? 1 : 0;
    for (int32_t t = 0; t < ns; ++t) {  // children precede parents
        int32_t lv = 0;
        for (int32_t q = P.ch_ptr[t]; q < P.ch_ptr[t + 1]; ++q) lv = std::max(lv, P.sn_level[P.ch[q]] + 1);
        P.sn_level[t] = lv;
        P.nlevels = std::max(P.nlevels, lv + 1);
    }

    // child -> parent relative maps of the CB rows
    P.rel_ptr.assign(ns + 1, 0);
    for (int32_t t = 0; t < ns; ++t) P.rel_ptr[t + 1] = P.rel_ptr[t] + (P.sn_f[t] - P.sn_p[t]);
    P.rel.resize(P.rel_ptr[ns]);
    for (int32_t t = 0; t < ns; ++t) {
        int32_t q = P.sn_parent[t];
        int32_t cb = P.sn_f[t] - P.sn_p[t];
        if (cb > 0 && q < 0) {
            msg = "internal: contribution block without a parent";
            return QDMF_ERR_INVALID_ARG;
        }
        for (int32_t i = 0; i < cb; ++i) {
            int32_t r = P.rows[P.sn_rowptr[t] + P.sn_p[t] + i];
            int32_t pos = find_pos(&P.rows[P.sn_rowptr[q]], P.sn_ptr[q], P.sn_p[q], P.sn_f[q], r);
            if (pos < 0) {
                msg = "internal: child row missing from parent front";
                return QDMF_ERR_INVALID_ARG;
            }
            P.rel[P.rel_ptr[t] + i] = pos;
        }
    }

    // entries of lower(K) by new column, with their front row positions and sources
    std::vector<int32_t> c2s(N);
    for (int32_t t = 0; t < ns; ++t)
        for (int32_t c = P.sn_ptr[t]; c < P.sn_ptr[t + 1]; ++c) c2s[c] = t;
    P.kcol_ptr.assign(N + 1, 0);
    for (int32_t c = 0; c < N; ++c) {
        int32_t old = P.perm[c];
        int64_t cnt = 1;
        for (int64_t e = xadj[old]; e < xadj[old + 1]; ++e) cnt += P.iperm[adj[e]] > c;
        P.kcol_ptr[c + 1] = P.kcol_ptr[c] + cnt;
    }
    const int64_t knnz = P.kcol_ptr[N];
    P.kloc.resize(knnz);
    P.kcl.resize(knnz);
    P.krow_old.resize(knnz);
    P.kcol_old.resize(knnz);
    {
        std::vector<int32_t> tmp;
        for (int32_t c = 0; c < N; ++c) {
            int32_t old = P.perm[c];
            tmp.clear();
            for (int64_t e = xadj[old]; e < xadj[old + 1]; ++e)
                if (P.iperm[adj[e]] > c) tmp.push_back(P.iperm[adj[e]]);
            std::sort(tmp.begin(), tmp.end());
            int32_t t = c2s[c];
            const int32_t* rr = &P.rows[P.sn_rowptr[t]];
            int64_t w = P.kcol_ptr[c];
            for (int64_t q = P.kcol_ptr[c]; q < P.kcol_ptr[c + 1]; ++q) P.kcl[q] = c - P.sn_ptr[t];
            P.kloc[w] = c - P.sn_ptr[t];
            P.krow_old[w] = old;
            P.kcol_old[w] = old;
            ++w;
            for (int32_t r : tmp) {
                int32_t pos = find_pos(rr, P.sn_ptr[t], P.sn_p[t], P.sn_f[t], r);
                if (pos < 0) {
                    msg = "internal: entry outside its front";
                    return QDMF_ERR_INVALID_ARG;
                }
                P.kloc[w] = pos;
                P.krow_old[w] = P.perm[r];
                P.kcol_old[w] = old;
                ++w;
            }
        }
    }
    if (mode == QDMF_AS) {
        P.ksrc.resize(knnz);
        for (int64_t e = 0; e < knnz; ++e) {
            int32_t a = P.krow_old[e], b = P.kcol_old[e];
            if (a == b) {
                P.ksrc[e] = a < n ? -1 - (int64_t)a : KSRC_ZERO;
            } else if (a < n && b < n) {  // an off-diagonal entry of Q
                const int32_t lo = std::min(a, b), hi = std::max(a, b);
                const int32_t* beg = &P.qri[0] + P.qcp[lo];
                const int32_t* end = &P.qri[0] + P.qcp[lo + 1];
                const int32_t* it = std::lower_bound(beg, end, hi);
                P.ksrc[e] = -1 - (int64_t)n - (P.qcp[lo] + (it - beg));
            } else {
                int32_t x = a < n ? a : b;  // primal index
                int32_t y = (a < n ? b : a) - n;
                const int32_t* beg = &P.ari[P.acp[x]];
                const int32_t* end = &P.ari[0] + P.acp[x + 1];
                const int32_t* it = std::lower_bound(beg, end, y);
                P.ksrc[e] = P.acp[x] + (it - beg);
            }
        }
    } else {
        // pairs (A_ij, A_kj) over the shared columns j, ascending
        P.kpair_ptr.assign(knnz + 1, 0);
        std::vector<int32_t> pr;
        for (int64_t e = 0; e < knnz; ++e) {
            int32_t i = P.krow_old[e], k = P.kcol_old[e];
            int64_t a = P.arp[i], ae = P.arp[i + 1], b = P.arp[k], be = P.arp[k + 1];
            while (a < ae && b < be) {
                int32_t ja = P.acol[P.are[a]], jb = P.acol[P.are[b]];
                if (ja < jb) ++a;
                else if (jb < ja) ++b;
                else {
                    pr.push_back(P.are[a]);
                    pr.push_back(P.are[b]);
                    ++a;
                    ++b;
                }
            }
            P.kpair_ptr[e + 1] = (int64_t)pr.size() / 2;
        }
        P.kpair = std::move(pr);
        // rows touching each entry, for the symmetric residual and the norm
        P.krs_ptr.assign(N + 1, 0);
        for (int64_t e = 0; e < knnz; ++e) {
            P.krs_ptr[P.krow_old[e] + 1]++;
            if (P.krow_old[e] != P.kcol_old[e]) P.krs_ptr[P.kcol_old[e] + 1]++;
        }
        for (int32_t i = 0; i < N; ++i) P.krs_ptr[i + 1] += P.krs_ptr[i];
        P.krs_ent.resize(P.krs_ptr[N]);
        P.krs_other.resize(P.krs_ptr[N]);
        std::vector<int64_t> fl(P.krs_ptr.begin(), P.krs_ptr.end() - 1);
        for (int64_t e = 0; e < knnz; ++e) {
            int32_t r = P.krow_old[e], c = P.kcol_old[e];
            P.krs_ent[fl[r]] = (int32_t)e;
            P.krs_other[fl[r]++] = c;
            if (r != c) {
                P.krs_ent[fl[c]] = (int32_t)e;
                P.krs_other[fl[c]++] = r;
            }
        }
        if (knnz > INT32_MAX) {
            msg = "lower(K) has more than 2^31-1 entries";
            return QDMF_ERR_INDEX_OVERFLOW;
        }
    }
    P.primal_new.assign(N, 0);
    if (mode == QDMF_AS)
        for (int32_t c = 0; c < N; ++c) P.primal_new[c] = P.perm[c] < n;

    // ----- systems of a batch (block-diagonal A): per column, per K index, index ranges,
    // pivot lists
    P.nsys = std::max(1, opt.nsys);
    P.sys_col.assign(n, 0);
    std::vector<int32_t> sys_row(m, 0);
    if (opt.nsys > 1) {
        for (int32_t q = 0; q < P.nsys; ++q) {
            for (int64_t j = opt.col_off[q]; j < opt.col_off[q + 1]; ++j) P.sys_col[j] = q;
            for (int64_t i = opt.row_off[q]; i < opt.row_off[q + 1]; ++i) sys_row[i] = q;
        }
    }
    P.sys_old.resize(N);
    for (int32_t v = 0; v < N; ++v)
        P.sys_old[v] = mode == QDMF_AS ? (v < n ? P.sys_col[v] : sys_row[v - n]) : sys_row[v];
    P.sys_new.resize(N);
    for (int32_t k = 0; k < N; ++k) P.sys_new[k] = P.sys_old[P.perm[k]];
    P.sys_rng.assign(4 * (size_t)P.nsys, 0);
    for (int32_t q = 0; q < P.nsys; ++q) {
        const int64_t c0 = opt.nsys > 1 ? opt.col_off[q] : 0, c1 = opt.nsys > 1 ? opt.col_off[q + 1] : n;
        const int64_t r0 = opt.nsys > 1 ? opt.row_off[q] : 0, r1 = opt.nsys > 1 ? opt.row_off[q + 1] : m;
        if (mode == QDMF_AS) {
            P.sys_rng[4 * q] = c0;
            P.sys_rng[4 * q + 1] = c1;
            P.sys_rng[4 * q + 2] = n + r0;
            P.sys_rng[4 * q + 3] = n + r1;
        } else {
            P.sys_rng[4 * q] = r0;
            P.sys_rng[4 * q + 1] = r1;
            P.sys_rng[4 * q + 2] = r1;
            P.sys_rng[4 * q + 3] = r1;
        }
    }
    P.sys_piv_ptr.assign(P.nsys + 1, 0);
    for (int32_t k = 0; k < N; ++k) P.sys_piv_ptr[P.sys_new[k] + 1]++;
    for (int32_t q = 0; q < P.nsys; ++q) P.sys_piv_ptr[q + 1] += P.sys_piv_ptr[q];
    P.sys_piv.resize(N);
    {
        std::vector<int64_t> fill(P.sys_piv_ptr.begin(), P.sys_piv_ptr.end() - 1);
        for (int32_t k = 0; k < N; ++k) P.sys_piv[fill[P.sys_new[k]]++] = k;
    }

    // ----- memory plan: dense square fronts, column-major, ld = f
    P.sn_ld.resize(ns);
    P.sn_off.resize(ns);
    P.sn_nwin.resize(ns);
    int64_t off = 0;
    for (int32_t t = 0; t < ns; ++t) {
        P.sn_ld[t] = P.sn_f[t];
        P.sn_off[t] = off;
        off += (int64_t)P.sn_f[t] * P.sn_ld[t];
        P.sn_nwin[t] = (P.sn_p[t] + NB - 1) / NB;
    }
    P.front_total = off;
    P.ub_off.resize(ns + 1);
    int64_t uo = 0;
    for (int32_t t = 0; t < ns; ++t) {
        P.ub_off[t] = uo;
        uo += P.sn_f[t] - P.sn_p[t];
    }
    P.ub_off[ns] = uo;
    P.ub_total = uo;
    // forward-solve gather lists: for every front row (indexed like rows[]), the children's
    // contribution-vector entries that land on it, children ascending
    P.fg_ptr.assign(P.sn_rowptr[ns] + 1, 0);
    for (int32_t t = 0; t < ns; ++t)
        for (int32_t q = P.ch_ptr[t]; q < P.ch_ptr[t + 1]; ++q) {
            const int32_t c = P.ch[q];
            for (int64_t a = P.rel_ptr[c]; a < P.rel_ptr[c + 1]; ++a) P.fg_ptr[P.sn_rowptr[t] + P.rel[a] + 1]++;
        }
    for (int64_t i = 0; i < P.sn_rowptr[ns]; ++i) P.fg_ptr[i + 1] += P.fg_ptr[i];
    P.fg_src.resize(P.fg_ptr.back());
    {
        std::vector<int64_t> fl(P.fg_ptr.begin(), P.fg_ptr.end() - 1);
        for (int32_t t = 0; t < ns; ++t)
            for (int32_t q = P.ch_ptr[t]; q < P.ch_ptr[t + 1]; ++q) {
                const int32_t c = P.ch[q];
                for (int64_t a = P.rel_ptr[c]; a < P.rel_ptr[c + 1]; ++a)
                    P.fg_src[fl[P.sn_rowptr[t] + P.rel[a]]++] = P.ub_off[c] + (a - P.rel_ptr[c]);
            }
    }

    // ----- solve level lists: per level the supernodes solved one per workgroup first, then
    // the big ones
    P.lvl_ptr.assign(P.nlevels + 1, 0);
    for (int32_t t = 0; t < ns; ++t) P.lvl_ptr[P.sn_level[t] + 1]++;
    for (int32_t l = 0; l < P.nlevels; ++l) P.lvl_ptr[l + 1] += P.lvl_ptr[l];
    P.lvl_sn.resize(ns);
    P.lvl_small.assign(P.nlevels, 0);
    P.lvl_wave.assign(P.nlevels, 0);
    {
        // a level that holds a front of at least split_solve_front pays the multi-workgroup
        // launches anyway (one diagonal solve and one update launch per SOLVE_BLOCK-pivot block
        // of its largest such front): its other fronts of at least SPLIT_JOIN_FRONT rows with no
        // more blocks join those launches rather than occupy one workgroup each for the level
        std::vector<int32_t> lvl_nb(P.nlevels, 0);
        for (int32_t t = 0; t < ns; ++t)
            if (P.sn_f[t] >= opt.split_solve_front)
                lvl_nb[P.sn_level[t]] = std::max(lvl_nb[P.sn_level[t]], (P.sn_p[t] + SOLVE_BLOCK - 1) / SOLVE_BLOCK);
        auto split = [&](int32_t t) {
            if (P.sn_f[t] >= opt.split_solve_front) return true;
            const int32_t nb = lvl_nb[P.sn_level[t]];
            return nb > 0 && P.sn_f[t] >= std::min(SPLIT_JOIN_FRONT, opt.split_solve_front) &&
                   (P.sn_p[t] + SOLVE_BLOCK - 1) / SOLVE_BLOCK <= nb;
        };
        // per level: fronts of at most 64 rows (one wavefront each), the other one-workgroup
        // supernodes, then the big ones
        std::vector<int64_t> fl(P.lvl_ptr.begin(), P.lvl_ptr.end() - 1);
        for (int pass = 0; pass < 3; ++pass)
            for (int32_t t = 0; t < ns; ++t) {
                const int cls = split(t) ? 2 : (P.sn_f[t] <= 64 ? 0 : 1);
                if (cls != pass) continue;
                P.lvl_sn[fl[P.sn_level[t]]++] = t;
                if (pass < 2) P.lvl_small[P.sn_level[t]]++;
                if (pass == 0) P.lvl_wave[P.sn_level[t]]++;
            }
    }
    // big supernodes: work-space rows and the launch sequence of each level
    P.yoff.assign(ns, -1);
    P.ytotal = 0;
    P.fwd_ptr.assign(P.nlevels + 1, 0);
    P.bwd_ptr.assign(P.nlevels + 1, 0);
    P.ppart_max = 0;
    auto chunks = [](int64_t rows) { return (int32_t)((rows + 255) / 256); };
    for (int32_t l = 0; l < P.nlevels; ++l) {
        std::vector<int32_t> big(P.lvl_sn.begin() + P.lvl_ptr[l] + P.lvl_small[l], P.lvl_sn.begin() + P.lvl_ptr[l + 1]);
        int32_t nbmax = 0;
        for (int32_t t : big) {
            P.yoff[t] = P.ytotal;
            P.ytotal += P.sn_f[t];
            nbmax = std::max(nbmax, (P.sn_p[t] + SOLVE_BLOCK - 1) / SOLVE_BLOCK);
        }
        auto add = [&](std::vector<SolveLaunch>& plan, int32_t kind, int64_t t0) {
            const int64_t cnt = (int64_t)P.stasks.size() - t0;
            if (cnt > 0) plan.push_back(SolveLaunch{kind, t0, cnt});
        };
        if (!big.empty()) {
            int64_t t0 = (int64_t)P.stasks.size();
            for (int32_t t : big)
                for (int32_t c = 0; c < chunks(P.sn_f[t]); ++c) P.stasks.push_back(Task{t, c, 0, 0});
            add(P.fwd_plan, S_GATHER, t0);
            for (int32_t j = 0; j < nbmax; ++j) {
                t0 = (int64_t)P.stasks.size();
                for (int32_t t : big)
                    if (SOLVE_BLOCK * j < P.sn_p[t]) P.stasks.push_back(Task{t, j, 0, 0});
                add(P.fwd_plan, S_FDIAG, t0);
                t0 = (int64_t)P.stasks.size();
                for (int32_t t : big)
                    if (SOLVE_BLOCK * j < P.sn_p[t]) {
                        const int32_t k1 = std::min(P.sn_p[t], SOLVE_BLOCK * (j + 1));
                        for (int32_t c = 0; c < chunks(P.sn_f[t] - k1); ++c) P.stasks.push_back(Task{t, j, c, 0});
                    }
                add(P.fwd_plan, S_FUPD, t0);
            }
            t0 = (int64_t)P.stasks.size();
            for (int32_t t : big)
                for (int32_t c = 0; c < chunks(P.sn_f[t]); ++c) P.stasks.push_back(Task{t, c, 0, 0});
            add(P.fwd_plan, S_FFIN, t0);
            // backward
            t0 = (int64_t)P.stasks.size();
            for (int32_t t : big)
                for (int32_t c = 0; c < chunks(P.sn_f[t]); ++c) P.stasks.push_back(Task{t, c, 0, 0});
            add(P.bwd_plan, S_BLOAD, t0);
            for (int32_t j = nbmax - 1; j >= 0; --j) {
                t0 = (int64_t)P.stasks.size();
                std::vector<std::pair<int32_t, int32_t>> range(big.size(), {0, 0});
                int32_t q = 0;
                for (size_t bi = 0; bi < big.size(); ++bi) {
                    const int32_t t = big[bi];
                    if (SOLVE_BLOCK * j >= P.sn_p[t]) continue;
                    const int32_t k1 = std::min(P.sn_p[t], SOLVE_BLOCK * (j + 1));
                    range[bi].first = q;
                    for (int32_t c = 0; c < chunks(P.sn_f[t] - k1); ++c) P.stasks.push_back(Task{t, j, c, q++});
                    range[bi].second = q - range[bi].first;
                }
                P.ppart_max = std::max<int64_t>(P.ppart_max, q);
                add(P.bwd_plan, S_BPART, t0);
                t0 = (int64_t)P.stasks.size();
                for (size_t bi = 0; bi < big.size(); ++bi)
                    if (SOLVE_BLOCK * j < P.sn_p[big[bi]])
                        P.stasks.push_back(Task{big[bi], j, range[bi].first, range[bi].second});
                add(P.bwd_plan, S_BDIAG, t0);
            }
            t0 = (int64_t)P.stasks.size();
            for (int32_t t : big)
                for (int32_t c = 0; c < chunks(P.sn_p[t]); ++c) P.stasks.push_back(Task{t, c, 0, 0});
            add(P.bwd_plan, S_BSTORE, t0);
        }
        P.fwd_ptr[l + 1] = (int64_t)P.fwd_plan.size();
        P.bwd_ptr[l + 1] = (int64_t)P.bwd_plan.size();
    }

    // ----- inverses of the 64-pivot diagonal blocks: for the levels solved by the
    // one-workgroup kernels with blocks of more than 8 pivots (levels whose fronts are all at
    // most 64 rows use one wavefront per supernode instead, and blocks of up to 8 pivots a
    // short serial sweep), and for every supernode of the multi-workgroup solves
    P.inv_off.assign(ns, -1);
    P.inv_total = 0;
    auto add_inv = [&](int32_t t) {
        const int32_t p = P.sn_p[t], nblk = (p + 63) / 64, nbl = p - 64 * (nblk - 1);
        if (p <= 0) return;
        P.inv_off[t] = P.inv_total;
        P.inv_total += 4096 * (int64_t)(nblk - 1) + (int64_t)nbl * nbl;
        for (int32_t j = 0; j < nblk; ++j) P.inv_tasks.push_back(Task{t, j, 0, 0});
    };
    for (int32_t l = 0; l < P.nlevels; ++l) {
        int32_t mf = 0, mp = 0;
        for (int64_t q = P.lvl_ptr[l]; q < P.lvl_ptr[l] + P.lvl_small[l]; ++q) {
            mf = std::max(mf, P.sn_f[P.lvl_sn[q]]);
            mp = std::max(mp, P.sn_p[P.lvl_sn[q]]);
        }
        if (mf > 64 && mp > 8)
            for (int64_t q = P.lvl_ptr[l]; q < P.lvl_ptr[l] + P.lvl_small[l]; ++q) add_inv(P.lvl_sn[q]);
        for (int64_t q = P.lvl_ptr[l] + P.lvl_small[l]; q < P.lvl_ptr[l + 1]; ++q) add_inv(P.lvl_sn[q]);
    }

    // ----- solve work per level (one pass, one rhs): L panel read once, vectors in and out
    P.lvl_solve_flops.assign(P.nlevels, 0.0);
    P.lvl_solve_bytes.assign(P.nlevels, 0.0);
    for (int32_t t = 0; t < ns; ++t) {
        const double f = P.sn_f[t], p = P.sn_p[t];
        const double lent = p * f - p * (p - 1) / 2;  // lower trapezoid of the panel
        P.lvl_solve_flops[P.sn_level[t]] += 2.0 * (lent - p) + p;
        P.lvl_solve_bytes[P.sn_level[t]] += 8.0 * lent + 8.0 * 3 * f;
    }

    // ----- factorisation launch plan, level by level
    P.tasks.clear();
    P.launches.clear();
    P.asm_child.clear();
    P.asm_col.clear();
    // algorithmic work per task (front dimensions as the kernels process them)
    auto task_work = [&](int32_t kind, int32_t npg, const Task& tk, double& fl, double& by) {
        const double f = P.sn_f[tk.s], p = P.sn_p[tk.s];
        if (kind == L_SMALL) {  // whole partial factorisation of the front + its assembly
            for (double k = 0; k < p; ++k) fl += (f - k - 1) * (f - k - 1 + 3);
            by += 8.0 * f * (f + 1) / 2;
            for (int32_t q = P.ch_ptr[tk.s]; q < P.ch_ptr[tk.s + 1]; ++q) {
                const double cb = P.sn_f[P.ch[q]] - P.sn_p[P.ch[q]];
                by += 8.0 * cb * (cb + 1) / 2 + 4.0 * cb;
            }
        } else if (kind == L_ASSEMBLE) {  // one front column: children's CB columns in, column out
            by += 8.0 * (f - tk.k0);
            for (int32_t q = tk.a; q < tk.a + tk.b; ++q) {
                const double cb = P.sn_f[P.asm_child[q]] - P.sn_p[P.asm_child[q]];
                by += 12.0 * (cb - P.asm_col[q]);
                fl += cb - P.asm_col[q];
            }
        } else if (kind == L_WINDOW) {  // eliminations restricted to the window columns
            const double k0 = tk.k0, k1 = std::min<double>(p, k0 + NB), ch = 64.0 * npg;
            const double panel = std::max(0.0, std::min(ch, f - k1 - ch * tk.a));
            const double rows = panel + (tk.a == 0 ? k1 - k0 : 0.0);
            for (double k = k0; k < k1; ++k) {
                const double below = panel + (tk.a == 0 ? k1 - k - 1 : 0.0);
                fl += below * (1 + 2 * (k1 - k - 1));
            }
            by += 16.0 * rows * (k1 - k0);
        } else if (kind == L_SYRK || kind == L_SYRK128) {  // one lower tile of the trailing update
            const double T = kind == L_SYRK ? 64.0 : 128.0;
            const double k0 = tk.k0 & SYRK_K0_MASK, cnt = ((tk.k0 >> SYRK_COUNT_SHIFT) & 7) + 1;
            const double k1 = std::min<double>(p, k0 + NB * cnt), nbw = k1 - k0;
            const double cmax = (tk.k0 & SYRK_NARROW) ? std::min<double>(p, k1 + NB) : f;
            const double r0 = k1 + T * tk.a, c0 = k1 + T * tk.b;
            const double nr = std::max(0.0, std::min(T, f - r0)), nc = std::max(0.0, std::min(T, cmax - c0));
            double lower = nr * nc;
            if (tk.a == tk.b) lower = nc * (nc + 1) / 2 + (nr - nc) * nc;
            fl += 2.0 * nbw * lower;
            by += 8.0 * (2 * lower + (nr + nc) * nbw);
        } else if (kind == L_FINALIZE) {  // one 64-column block of one window: read + write
            const double nc = std::min<double>(NB, p - tk.k0), nr = std::min<double>(NB, p - (double)tk.a * NB);
            by += tk.a * NB == tk.k0 ? 16.0 * nc * (nc - 1) / 2 : 16.0 * nc * nr;
        }
    };
    auto add_launch = [&](int32_t kind, int32_t lvl, int64_t t0, int32_t lds, int32_t maxf, int32_t npg = 0) {
        int64_t cnt = (int64_t)P.tasks.size() - t0;
        if (cnt > 0) {
            Launch L{kind, lvl, t0, cnt, lds, maxf};
            L.npg = npg;
            for (int64_t q = t0; q < t0 + cnt; ++q) task_work(kind, npg, P.tasks[q], L.flops, L.bytes);
            P.launches.push_back(L);
        }
    };
    for (int32_t l = 0; l < P.nlevels; ++l) {
        std::vector<int32_t> small, large;
        for (int64_t q = P.lvl_ptr[l]; q < P.lvl_ptr[l + 1]; ++q) {
            int32_t t = P.lvl_sn[q];
            (P.sn_f[t] <= opt.small_front ? small : large).push_back(t);
        }
        int64_t t0 = (int64_t)P.tasks.size();
        int32_t mf = 0;
        for (int32_t t : small) {
            P.tasks.push_back(Task{t, 0, 0, 0});
            mf = std::max(mf, P.sn_f[t]);
        }
        add_launch(L_SMALL, l, t0, 0, mf);
        if (large.empty()) continue;
        t0 = (int64_t)P.tasks.size();
        mf = 0;
        for (int32_t t : large) {
            // (child, child CB column) pairs of each parent column, children ascending
            std::vector<std::vector<std::pair<int32_t, int32_t>>> lists(P.sn_f[t]);
            for (int32_t q = P.ch_ptr[t]; q < P.ch_ptr[t + 1]; ++q) {
                const int32_t c = P.ch[q];
                const int32_t cb = P.sn_f[c] - P.sn_p[c];
                for (int32_t i = 0; i < cb; ++i) lists[P.rel[P.rel_ptr[c] + i]].push_back({c, i});
            }
            for (int32_t j = 0; j < P.sn_f[t]; ++j) {
                const int32_t a = (int32_t)P.asm_child.size();
                for (auto& pr : lists[j]) {
                    P.asm_child.push_back(pr.first);
                    P.asm_col.push_back(pr.second);
                }
                P.tasks.push_back(Task{t, j, a, (int32_t)lists[j].size()});
            }
            mf = std::max(mf, P.sn_f[t]);
        }
        if (mf > 16384) {
            msg = "front order above 16384 is not supported";
            return QDMF_ERR_UNSUPPORTED;
        }
        add_launch(L_ASSEMBLE, l, t0, mf * 8, mf);
        int32_t maxwin = 0;
        for (int32_t t : large) maxwin = std::max(maxwin, P.sn_nwin[t]);
        for (int32_t w = 0; w < maxwin; ++w) {
            // panel rows per workgroup: 64 * npg with npg <= 1 (more rows per workgroup make
            // every pivot step of the window longer; more workgroups repeat the decisions)
            int32_t npg = 0;
            for (int32_t t : large)
                if (w < P.sn_nwin[t]) {
                    const int32_t k1 = std::min(P.sn_p[t], (w + 1) * NB);
                    npg = std::max(npg, std::min(1, (P.sn_f[t] - k1 + 63) / 64));
                }
            t0 = (int64_t)P.tasks.size();
            mf = 0;
            for (int32_t t : large)
                if (w < P.sn_nwin[t]) {
                    const int32_t k1 = std::min(P.sn_p[t], (w + 1) * NB);
                    const int32_t rows_below = P.sn_f[t] - k1;
                    const int32_t nchunk = npg ? std::max(1, (rows_below + 64 * npg - 1) / (64 * npg)) : 1;
                    for (int32_t c = 0; c < nchunk; ++c) P.tasks.push_back(Task{t, w * NB, c, 0});
                    mf = std::max(mf, P.sn_f[t]);
                }
            add_launch(L_WINDOW, l, t0, 0, mf, npg);
            // Schur update after window w.  A front of at least syrk_group_front rows takes its
            // windows in groups of syrk_group: inside a group, only the next window's columns
            // receive the update of the group's windows so far (what that window's
            // factorisation needs); after the group's last window, the rest of the trailing
            // matrix receives the update of all its windows at once, so each trailing entry is
            // read and written once per group instead of once per window.
            // the full updates of trailing matrices of at least syrk_tile_front rows go in 128 x 128
            // tiles (their own launch, before the one of the 64 x 64 tiles)
            auto group_of = [&](int32_t t, int32_t& g, int32_t& last) {
                const bool grouped = opt.syrk_group_front > 0 && P.sn_f[t] >= opt.syrk_group_front;
                const int32_t G = grouped ? opt.syrk_group : 1;
                g = (w / G) * G;
                last = std::min(g + G, P.sn_nwin[t]) - 1;
            };
            auto wide = [&](int32_t t, int32_t last) {
                const int32_t k1 = std::min(P.sn_p[t], (w + 1) * NB);
                return w == last && opt.syrk_tile_front > 0 && P.sn_f[t] - k1 >= opt.syrk_tile_front;
            };
            // Lookahead (fronts of order >= lookahead_front): a full update is split by columns.
            // Its tiles over the next group's pivot columns stay on the main stream (the next
            // windows need them); the tiles beyond them go to the second stream and run while
            // the next group's windows and narrow updates run, which touch only their own
            // columns.  The next full update of that front overlaps those columns, so the
            // launch that holds it waits for the second stream first.
            auto split_cols = [&](int32_t t, int32_t T) {  // tile columns kept on the main stream
                if (opt.lookahead_front <= 0 || P.sn_f[t] < opt.lookahead_front) return INT32_MAX;
                const int32_t Gn = (opt.syrk_group_front > 0 && P.sn_f[t] >= opt.syrk_group_front) ? opt.syrk_group : 1;
                const int32_t k1 = std::min(P.sn_p[t], (w + 1) * NB);
                const int32_t next_cols = std::min(P.sn_p[t], k1 + Gn * NB) - k1;
                return (next_cols + T - 1) / T;
            };
            std::vector<Task> ta[2], tb[2];  // [main, second stream] x [128, 64 tiles]
            int64_t nmix[2] = {0, 0};
            bool full_la = false;  // the main-stream part holds a full update of a lookahead front
            for (int pass = 0; pass < 2; ++pass)  // fronts of order >= f_mix first
            for (int32_t t : large)
                if (w < P.sn_nwin[t] && (P.sn_f[t] >= opt.f_mix) == (pass == 0)) {
                    int32_t g, last;
                    group_of(t, g, last);
                    if (!wide(t, last)) continue;
                    const int32_t k1 = std::min(P.sn_p[t], (w + 1) * NB);
                    const int32_t R = (P.sn_f[t] - k1 + 127) / 128;
                    const int32_t code = g * NB | (w - g) << SYRK_COUNT_SHIFT;
                    const int32_t nA = split_cols(t, 128);
                    for (int32_t bj = 0; bj < R; ++bj)
                        for (int32_t bi = bj; bi < R; ++bi) {
                            const int st = bj < nA ? 0 : 1;
                            ta[st].push_back(Task{t, code, bi, bj});
                            if (pass == 0) ++nmix[st];
                            if (st == 0 && nA != INT32_MAX) full_la = true;
                        }
                }
            for (int32_t t : large)
                if (w < P.sn_nwin[t]) {
                    int32_t g, last;
                    group_of(t, g, last);
                    if (wide(t, last)) continue;
                    const int32_t k1 = std::min(P.sn_p[t], (w + 1) * NB);
                    const int32_t R = (P.sn_f[t] - k1 + 63) / 64;
                    const int32_t code = g * NB | (w - g) << SYRK_COUNT_SHIFT;
                    if (w < last) {  // window w + 1 is whole or partial, its columns start at k1
                        for (int32_t bi = 0; bi < R; ++bi) tb[0].push_back(Task{t, code | SYRK_NARROW, bi, 0});
                    } else {
                        const int32_t nA = split_cols(t, 64);
                        for (int32_t bj = 0; bj < R; ++bj)
                            for (int32_t bi = bj; bi < R; ++bi) {
                                const int st = bj < nA ? 0 : 1;
                                tb[st].push_back(Task{t, code, bi, bj});
                                if (st == 0 && nA != INT32_MAX) full_la = true;
                            }
                    }
                }
            for (int st = 0; st < 2; ++st) {
                t0 = (int64_t)P.tasks.size();
                P.tasks.insert(P.tasks.end(), ta[st].begin(), ta[st].end());
                add_launch(L_SYRK128, l, t0, 0, mf);
                if (!P.launches.empty() && P.launches.back().kind == L_SYRK128 && P.launches.back().task0 == t0) {
                    P.launches.back().nmix = nmix[st];
                    P.launches.back().stream = (int8_t)st;
                    P.launches.back().wait = (int8_t)(st == 0 && full_la);
                }
                t0 = (int64_t)P.tasks.size();
                P.tasks.insert(P.tasks.end(), tb[st].begin(), tb[st].end());
                add_launch(L_SYRK, l, t0, 0, mf);
                if (!P.launches.empty() && P.launches.back().kind == L_SYRK && P.launches.back().task0 == t0) {
                    P.launches.back().stream = (int8_t)st;
                    P.launches.back().wait = (int8_t)(st == 0 && full_la);
                }
            }
        }
        // The level's last update may sit on the second stream; nothing of this level follows
        // it, so it moves to the main stream behind a join (and can take the finalize tasks).
        if (!P.launches.empty() && P.launches.back().level == l && P.launches.back().stream == 1) {
            P.launches.back().stream = 0;
            P.launches.back().wait = 1;
        }
        t0 = (int64_t)P.tasks.size();
        for (int32_t t : large)
            for (int32_t c = 0; c < P.sn_nwin[t]; ++c)
                for (int32_t w = c; w < P.sn_nwin[t]; ++w) P.tasks.push_back(Task{t, c * NB, w, 0});
        // The level's last trailing update touches only rows and columns past every pivot of
        // its fronts, and the finalize tasks only pivot rows and columns: both run in one
        // launch when there is such an update.
        if (!P.launches.empty() && (P.launches.back().kind == L_SYRK || P.launches.back().kind == L_SYRK128) &&
            P.launches.back().level == l) {
            Launch& L = P.launches.back();
            L.fin0 = t0;
            L.nfin = (int64_t)P.tasks.size() - t0;
            for (int64_t q = t0; q < t0 + L.nfin; ++q) task_work(L_FINALIZE, 0, P.tasks[q], L.flops, L.bytes);
        } else {
            add_launch(L_FINALIZE, l, t0, 0, 0);
        }
    }
    return 0;
}

}  // namespace qdmf
