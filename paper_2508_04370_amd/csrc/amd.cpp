// Approximate minimum degree ordering (Amestoy, Davis & Duff, SIAM J. Matrix Anal. Appl.
// 17(4), 1996), written from the published description: quotient graph of variables and
// elements, element absorption, approximate external degrees
//   d_i = min( n_left - |i|,  d_i_old + |L_p \ i|,  |A_i| + |L_p \ i| + sum_{e in E_i, e != p} |L_e \ L_p| ),
// aggressive absorption of elements contained in the new element, supervariable detection
// by hashing, mass elimination, and dense rows postponed to the end.
// The paper orders with nested dissection (Section 4.2); its configs name minimum degree for
// the random and staircase problems, which is what this provides.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "plan.hpp"

namespace qdmf {

namespace {
enum : int8_t { VAR = 0, ELEM = 1, DEAD = 2 };
}

void amd_order(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
               std::vector<int32_t>& order) {
    order.clear();
    order.reserve(N);
    if (N == 0) return;
    std::vector<std::vector<int32_t>> A(N), E(N), L(N), members(N);
    std::vector<int64_t> nv(N, 1), deg(N, 0), esize(N, 0), w(N, 0);
    std::vector<int32_t> mark(N, 0), wtag(N, 0);
    std::vector<int8_t> st(N, VAR);

    // dense rows are taken out and ordered last
    const double dense_thr = std::max(16.0, 10.0 * std::sqrt((double)N));
    std::vector<int32_t> dense;
    std::vector<char> isdense(N, 0);
    if (N > 64) {
        for (int32_t i = 0; i < N; ++i)
            if ((double)(xadj[i + 1] - xadj[i]) > dense_thr) {
                isdense[i] = 1;
                st[i] = DEAD;
                dense.push_back(i);
            }
    }
    const int64_t neff = N - (int64_t)dense.size();
    for (int32_t i = 0; i < N; ++i) {
        if (isdense[i]) continue;
        for (int64_t e = xadj[i]; e < xadj[i + 1]; ++e)
            if (!isdense[adj[e]] && adj[e] != i) A[i].push_back(adj[e]);
        deg[i] = (int64_t)A[i].size();
    }

    // degree buckets (doubly linked lists)
    std::vector<int32_t> head(N + 1, -1), nxt(N, -1), prv(N, -1);
    std::vector<char> inb(N, 0);
    int64_t mindeg = N;
    auto bucket_of = [&](int32_t i) { return (int32_t)std::min<int64_t>(std::max<int64_t>(deg[i], 0), N); };
    auto ins = [&](int32_t i) {
        int32_t d = bucket_of(i);
        nxt[i] = head[d];
        prv[i] = -1;
        if (head[d] >= 0) prv[head[d]] = i;
        head[d] = i;
        inb[i] = 1;
        if (d < mindeg) mindeg = d;
    };
    auto rem = [&](int32_t i) {
        if (!inb[i]) return;
        int32_t d = bucket_of(i);
        if (prv[i] >= 0) nxt[prv[i]] = nxt[i];
        else head[d] = nxt[i];
        if (nxt[i] >= 0) prv[nxt[i]] = prv[i];
        inb[i] = 0;
    };
    for (int32_t i = N - 1; i >= 0; --i)
        if (st[i] == VAR) ins(i);

    std::vector<int32_t> seq;  // principal pivots in elimination order
    seq.reserve(N);
    int32_t tag = 0, wstamp = 0;
    int64_t nel = 0;
    std::vector<int32_t> Lp;
    std::vector<std::pair<uint64_t, int32_t>> hashes;

    while (nel < neff) {
        while (mindeg <= N && head[mindeg] < 0) ++mindeg;
        const int32_t p = head[mindeg];
        rem(p);
        seq.push_back(p);
        nel += nv[p];

        // new element L_p = (A_p U union of L_e over e in E_p) \ {p}; absorb those e
        ++tag;
        mark[p] = tag;
        Lp.clear();
        int64_t degme = 0;
        for (int32_t e : E[p]) {
            if (st[e] != ELEM) continue;
            for (int32_t i : L[e])
                if (st[i] == VAR && mark[i] != tag) {
                    mark[i] = tag;
                    Lp.push_back(i);
                    degme += nv[i];
                }
            st[e] = DEAD;
            std::vector<int32_t>().swap(L[e]);
        }
        for (int32_t i : A[p])
            if (st[i] == VAR && mark[i] != tag) {
                mark[i] = tag;
                Lp.push_back(i);
                degme += nv[i];
            }
        std::vector<int32_t>().swap(A[p]);
        std::vector<int32_t>().swap(E[p]);
        st[p] = ELEM;

        // prune the lists of the variables in L_p
        for (int32_t i : Lp) {
            rem(i);
            auto& Ei = E[i];
            size_t q = 0;
            for (int32_t e : Ei)
                if (st[e] == ELEM) Ei[q++] = e;
            Ei.resize(q);
            Ei.push_back(p);
            auto& Ai = A[i];
            q = 0;
            for (int32_t j : Ai)
                if (st[j] == VAR && mark[j] != tag) Ai[q++] = j;
            Ai.resize(q);
        }
        // |L_e \ L_p| for the other elements adjacent to L_p
        ++wstamp;
        for (int32_t i : Lp)
            for (int32_t e : E[i]) {
                if (e == p) continue;
                if (wtag[e] != wstamp) {
                    wtag[e] = wstamp;
                    w[e] = esize[e];
                }
                w[e] -= nv[i];
            }
        // approximate degrees, aggressive absorption, mass elimination
        size_t keep = 0;
        for (size_t t = 0; t < Lp.size(); ++t) {
            int32_t i = Lp[t];
            int64_t ext = 0;
            auto& Ei = E[i];
            size_t q = 0;
            for (int32_t e : Ei) {
                if (e == p) {
                    Ei[q++] = e;
                    continue;
                }
                if (st[e] != ELEM) continue;
                if (w[e] <= 0) {  // L_e within L_p: absorb e into p
                    st[e] = DEAD;
                    std::vector<int32_t>().swap(L[e]);
                    continue;
                }
                ext += w[e];
                Ei[q++] = e;
            }
            Ei.resize(q);
            for (int32_t j : A[i]) ext += nv[j];
            if (ext == 0) {  // only adjacent to p: eliminate together with p
                st[i] = DEAD;
                members[p].push_back(i);
                members[p].insert(members[p].end(), members[i].begin(), members[i].end());
                std::vector<int32_t>().swap(members[i]);
                nel += nv[i];
                degme -= nv[i];
                nv[i] = 0;
                std::vector<int32_t>().swap(A[i]);
                std::vector<int32_t>().swap(E[i]);
                continue;
            }
            deg[i] = std::min(deg[i] + degme - nv[i], ext + degme - nv[i]);
            Lp[keep++] = i;
        }
        Lp.resize(keep);
        for (int32_t i : Lp) {
            int64_t d = std::min<int64_t>(deg[i], neff - nel - nv[i]);
            deg[i] = std::max<int64_t>(d, 0);
        }

        // supervariables: equal (A_i, E_i) sets among the variables of L_p
        hashes.clear();
        for (int32_t i : Lp) {
            std::sort(A[i].begin(), A[i].end());
            std::sort(E[i].begin(), E[i].end());
            uint64_t h = 1469598103934665603ull;
            for (int32_t j : A[i]) h = (h ^ (uint64_t)(j + 1)) * 1099511628211ull;
            h = (h ^ 0x9e3779b97f4a7c15ull) * 1099511628211ull;
            for (int32_t e : E[i]) h = (h ^ (uint64_t)(e + 1)) * 1099511628211ull;
            hashes.push_back({h, i});
        }
        std::sort(hashes.begin(), hashes.end());
        for (size_t a = 0; a < hashes.size();) {
            size_t b = a;
            while (b < hashes.size() && hashes[b].first == hashes[a].first) ++b;
            for (size_t x = a; x < b; ++x) {
                int32_t i = hashes[x].second;
                if (st[i] != VAR) continue;
                for (size_t y = x + 1; y < b; ++y) {
                    int32_t j = hashes[y].second;
                    if (st[j] != VAR) continue;
                    if (A[i] == A[j] && E[i] == E[j]) {
                        nv[i] += nv[j];
                        deg[i] -= nv[j];
                        if (deg[i] < 0) deg[i] = 0;
                        members[i].push_back(j);
                        members[i].insert(members[i].end(), members[j].begin(), members[j].end());
                        std::vector<int32_t>().swap(members[j]);
                        st[j] = DEAD;
                        nv[j] = 0;
                        std::vector<int32_t>().swap(A[j]);
                        std::vector<int32_t>().swap(E[j]);
                    }
                }
            }
            a = b;
        }
        // finish element p and reinsert its variables
        auto& Lpe = L[p];
        Lpe.clear();
        int64_t es = 0;
        for (int32_t i : Lp)
            if (st[i] == VAR) {
                Lpe.push_back(i);
                es += nv[i];
                ins(i);
            }
        esize[p] = es;
    }
    for (int32_t p : seq) {
        order.push_back(p);
        for (int32_t j : members[p]) order.push_back(j);
    }
    for (int32_t d : dense) order.push_back(d);
}

}  // namespace qdmf
