// Geometric nested dissection for problems whose rows live on an nx x ny x nz grid
// (Section 4.2 orders with nested dissection; the configs coupled on a grid name it).
// A box of rows is split across its longest side by a slab of rows; in the augmented
// system a primal column goes to the side that holds all of its rows, otherwise to the
// separator (so dense columns end up in the top separator, i.e. last).  The slab is two
// planes thick for the normal equations (rows are coupled at grid distance 2 through a
// shared column) and one plane for the augmented system.  Separators are ordered after
// both halves; boxes of at most 512 rows are ordered by minimum degree.
#include <algorithm>
#include <vector>

#include "../../include/qdmf.h"
#include "plan.hpp"

namespace qdmf {

namespace {

struct Ctx {
    const Plan* P;
    int g[3];
    int thick;
    const std::vector<int64_t>* xadj;
    const std::vector<int32_t>* adj;
    std::vector<int32_t>* out;
    std::vector<int32_t> local;  // node -> local index (scratch)
};

void order_leaf(Ctx& C, const std::vector<int32_t>& nodes) {
    // minimum degree on the induced subgraph
    const auto& xadj = *C.xadj;
    const auto& adj = *C.adj;
    int32_t k = (int32_t)nodes.size();
    for (int32_t i = 0; i < k; ++i) C.local[nodes[i]] = i;
    std::vector<int64_t> sx(k + 1, 0);
    std::vector<int32_t> sa;
    for (int32_t i = 0; i < k; ++i) {
        int32_t v = nodes[i];
        for (int64_t e = xadj[v]; e < xadj[v + 1]; ++e)
            if (C.local[adj[e]] >= 0) sa.push_back(C.local[adj[e]]);
        sx[i + 1] = (int64_t)sa.size();
    }
    std::vector<int32_t> ord;
    amd_order(k, sx, sa, ord);
    for (int32_t i : ord) C.out->push_back(nodes[i]);
    for (int32_t v : nodes) C.local[v] = -1;
}

void dissect(Ctx& C, std::vector<int32_t>& rows, std::vector<int32_t>& cols, int lo[3], int hi[3]) {
    const Plan& P = *C.P;
    int64_t vol = (int64_t)(hi[0] - lo[0]) * (hi[1] - lo[1]) * (hi[2] - lo[2]);
    int d = 0;
    for (int a = 1; a < 3; ++a)
        if (hi[a] - lo[a] > hi[d] - lo[d]) d = a;
    if (vol <= 512 || hi[d] - lo[d] <= C.thick + 1) {
        std::vector<int32_t> nodes(cols);
        for (int32_t r : rows) nodes.push_back(P.mode == QDMF_AS ? P.n + r : r);
        order_leaf(C, nodes);
        return;
    }
    int mid = (lo[d] + hi[d] - C.thick) / 2;
    auto coord = [&](int32_t r) {
        int x = r % C.g[0], y = (r / C.g[0]) % C.g[1], z = r / (C.g[0] * C.g[1]);
        return d == 0 ? x : (d == 1 ? y : z);
    };
    auto side = [&](int32_t r) {
        int c = coord(r);
        return c < mid ? 0 : (c >= mid + C.thick ? 1 : 2);
    };
    std::vector<int32_t> rl, rr, rs, cl, cr, csep;
    for (int32_t r : rows) {
        int s = side(r);
        (s == 0 ? rl : (s == 1 ? rr : rs)).push_back(r);
    }
    for (int32_t j : cols) {  // augmented system: primal columns follow their rows
        bool l = false, rgt = false;
        for (int64_t e = P.acp[j]; e < P.acp[j + 1]; ++e) {
            int s = side(P.ari[e]);
            l |= s == 0;
            rgt |= s == 1;
        }
        if (l && !rgt) cl.push_back(j);
        else if (rgt && !l) cr.push_back(j);
        else csep.push_back(j);
    }
    std::vector<int32_t>().swap(rows);
    std::vector<int32_t>().swap(cols);
    int lo2[3] = {lo[0], lo[1], lo[2]}, hi2[3] = {hi[0], hi[1], hi[2]};
    hi2[d] = mid;
    dissect(C, rl, cl, lo, hi2);
    lo2[d] = mid + C.thick;
    dissect(C, rr, cr, lo2, hi);
    // separator last; rows are grid ids, mapped to K nodes
    std::vector<int32_t> nodes;
    for (int32_t j : csep) nodes.push_back(j);
    for (int32_t r : rs) nodes.push_back(P.mode == QDMF_AS ? P.n + r : r);
    order_leaf(C, nodes);
}

}  // namespace

void grid_nd_order(const Plan& P, const int grid[3], const std::vector<int64_t>& xadj,
                   const std::vector<int32_t>& adj, std::vector<int32_t>& order) {
    Ctx C;
    C.P = &P;
    for (int a = 0; a < 3; ++a) C.g[a] = grid[a];
    C.thick = P.mode == QDMF_AS ? 1 : 2;
    C.xadj = &xadj;
    C.adj = &adj;
    C.out = &order;
    C.local.assign(P.N, -1);
    order.clear();
    order.reserve(P.N);
    std::vector<int32_t> rows(P.m), cols;
    for (int32_t r = 0; r < P.m; ++r) rows[r] = r;
    if (P.mode == QDMF_AS) {
        cols.resize(P.n);
        for (int32_t j = 0; j < P.n; ++j) cols[j] = j;
    }
    int lo[3] = {0, 0, 0}, hi[3] = {grid[0], grid[1], grid[2]};
    dissect(C, rows, cols, lo, hi);
}

}  // namespace qdmf
