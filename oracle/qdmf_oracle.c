/*
 * Reference (oracle) implementation: plain FP64 multifrontal LDL^T with the paper's
 * Bunch-Kaufman-variant pivoting and static/dynamic regularisation.
 *
 * TEST INFRASTRUCTURE ONLY (see qdmf_oracle.h).  Written for a reader checking it
 * against the paper: every step names the section or equation it follows.  No blocking,
 * no fusion; right-looking, one pivot at a time, full symmetric dense fronts.
 *
 * Readings of points the paper leaves open (also listed in the design notes):
 *  - the input is Theta; 1/Theta_j is one IEEE division;
 *  - NE with rho: theta~ = 1/(1/Theta + rho), K = A diag(theta~) A^T + delta I;
 *  - static regularisation s_k (-rho for primal, +delta for dual rows) is added to the
 *    pivot after the pivot tests (Section 4.5);
 *  - the lift uses ||K_static||_1 of the whole matrix;
 *  - the pivot window is nb consecutive pivot columns of the supernode; the presort swap
 *    happens before every pivot choice; ties go to the lowest position;
 *  - gamma_r is the largest off-diagonal magnitude of column r among the window's
 *    uneliminated rows (includes |F_kr|);
 *  - Proposition 3 is applied to 1x1 pivots against the window's same-sign columns with
 *    the regularised diagonal |F_jj + s_j| (zero denominators skipped and counted);
 *  - a pivot that still has the wrong sign is flipped to sign sigma_k with magnitude
 *    max(|d|, beta, eps*||K||_1) (Section 4.6: signs must not change);
 *  - a 2x2 pivot with zero determinant falls back to a lifted 1x1 pivot;
 *  - quadratic programs (AS only): the (1,1) block is -(Q + Theta^-1 + rho I); Q's
 *    off-diagonal couplings join the pattern, and the pivot signs and shifts are those of
 *    the LP (Q positive semidefinite keeps the matrix quasidefinite).
 */
#include "qdmf_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

struct orc_sym {
    int m, n, mode, N;
    /* lower pattern of K (incl. diagonal), ORIGINAL numbering, CSC, rows sorted */
    int64_t* kp;
    int32_t* ki;
    int32_t* perm;   /* new -> old */
    int32_t* iperm;  /* old -> new */
    int32_t* parent; /* column elimination tree, new numbering, -1 for roots */
    int64_t* colcount;
    int nsuper;
    int32_t* snptr;
    int32_t* snparent;
    int32_t* col2sn;
    int64_t* rowptr; /* front row lists, new numbering, sorted */
    int32_t* rows;
    int64_t nnzL;
    int64_t maxfront;
    double flops;
    /* copy of A pattern (needed by the numeric phase) */
    int64_t* acp;
    int32_t* ari;
    /* quadratic programs: lower triangle of Q (n x n CSC), NULL for an LP */
    int64_t* qcp;
    int32_t* qri;
};

struct orc_num {
    const orc_sym* S;
    double knorm;
    double rho, delta;
    double* theta; /* copy */
    double* aval;  /* copy */
    double* qval;  /* copy of Q's lower values, NULL for an LP */
    double* kval;  /* K0 values on S->kp/ki (original numbering) */
    int64_t* Lptr; /* per supernode offset of its f x p panel (ld = f) */
    double* L;
    double* d;     /* by position (new numbering) */
    double* doff;
    int8_t* ptype;
    double* edyn;
    int8_t* eflag;  /* by position: which dynamic regularisation fired (ORC_EF_* bits) */
    int32_t* lperm; /* by position: local original position within the supernode */
    orc_stats st;
    orc_opts opts;
};

void orc_default_opts(orc_opts* o) {
    o->nb = 64;
    o->alpha = (1.0 + sqrt(17.0)) / 8.0;
    o->eps_lift = 2.220446049250313e-16; /* 2^-52 */
    o->presort = 1;
    o->max_refine = 2;
    o->target_berr = 1e-12;
    o->tau_big = 1e-8;
}

/* ------------------------------------------------------------------ small helpers */

typedef struct {
    int32_t* v;
    int n, cap;
} ivec;

static void iv_push(ivec* a, int32_t x) {
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 8;
        a->v = (int32_t*)realloc(a->v, sizeof(int32_t) * (size_t)a->cap);
    }
    a->v[a->n++] = x;
}

static int cmp_i32(const void* a, const void* b) {
    int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
    return (x > y) - (x < y);
}

/* ------------------------------------------------------------------ K pattern (Section 3) */

/* Full adjacency (no diagonal) of K in original numbering: AS nodes 0..n-1 are the primal
 * variables x_j, n..n+m-1 the dual variables y_i, with x_j -- y_i iff A_ij != 0
 * (equation (augsys)).  NE nodes are the rows of A, with i -- k iff some column of A has
 * both (equation (normeq)). */
static ivec* build_adjacency(int m, int n, const int64_t* cp, const int32_t* ri, int mode,
                             const int64_t* qcp, const int32_t* qri, int* Nout) {
    int N = (mode == ORC_AS) ? n + m : m;
    ivec* adj = (ivec*)calloc((size_t)N, sizeof(ivec));
    if (mode == ORC_AS) {
        for (int j = 0; j < n; ++j)
            for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
                iv_push(&adj[j], n + ri[e]);
                iv_push(&adj[n + ri[e]], j);
            }
        /* quadratic programs: x_j -- x_k iff Q_kj != 0, k != j */
        if (qcp)
            for (int j = 0; j < n; ++j)
                for (int64_t e = qcp[j]; e < qcp[j + 1]; ++e)
                    if (qri[e] != j) {
                        iv_push(&adj[j], qri[e]);
                        iv_push(&adj[qri[e]], j);
                    }
    } else {
        for (int j = 0; j < n; ++j)
            for (int64_t a = cp[j]; a < cp[j + 1]; ++a)
                for (int64_t b = cp[j]; b < cp[j + 1]; ++b)
                    if (a != b) iv_push(&adj[ri[a]], ri[b]);
    }
    for (int v = 0; v < N; ++v) { /* sort + unique */
        qsort(adj[v].v, (size_t)adj[v].n, sizeof(int32_t), cmp_i32);
        int w = 0;
        for (int t = 0; t < adj[v].n; ++t)
            if (w == 0 || adj[v].v[w - 1] != adj[v].v[t]) adj[v].v[w++] = adj[v].v[t];
        adj[v].n = w;
    }
    *Nout = N;
    return adj;
}

/* ------------------------------------------------------------------ minimum degree (Section 4.2) */

/* The paper orders with a fill-reducing heuristic computed once.  The oracle uses plain
 * minimum degree on the explicit elimination graph: repeatedly eliminate the uneliminated
 * node of smallest current degree (lowest index on ties) and join its neighbours into a
 * clique.  Slow but obviously correct. */
typedef struct {
    int32_t deg, v;
} hent;

static int hless(hent a, hent b) { return a.deg < b.deg || (a.deg == b.deg && a.v < b.v); }

static void hpush(hent* h, int64_t* hn, hent x) {
    int64_t i = (*hn)++;
    h[i] = x;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (!hless(h[i], h[p])) break;
        hent t = h[i]; h[i] = h[p]; h[p] = t;
        i = p;
    }
}

static hent hpop(hent* h, int64_t* hn) {
    hent top = h[0];
    h[0] = h[--(*hn)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, s = i;
        if (l < *hn && hless(h[l], h[s])) s = l;
        if (r < *hn && hless(h[r], h[s])) s = r;
        if (s == i) break;
        hent t = h[i]; h[i] = h[s]; h[s] = t;
        i = s;
    }
    return top;
}

static void min_degree(int N, ivec* adj, int32_t* order) {
    int64_t hcap = N + 16, hn = 0;
    hent* h = (hent*)malloc(sizeof(hent) * (size_t)hcap);
    char* done = (char*)calloc((size_t)N, 1);
    int32_t* tmp = NULL;
    int tcap = 0;
    for (int v = 0; v < N; ++v) {
        hent e = {adj[v].n, v};
        hpush(h, &hn, e);
    }
    for (int step = 0; step < N; ++step) {
        hent e;
        do {
            e = hpop(h, &hn);
        } while (done[e.v] || e.deg != adj[e.v].n);
        int v = e.v;
        order[step] = v;
        done[v] = 1;
        ivec* av = &adj[v];
        for (int t = 0; t < av->n; ++t) {
            int u = av->v[t];
            ivec* au = &adj[u];
            /* new adj(u) = (adj(u) U adj(v)) \ {u, v}, sorted merge */
            int need = au->n + av->n;
            if (need > tcap) {
                tcap = need;
                tmp = (int32_t*)realloc(tmp, sizeof(int32_t) * (size_t)tcap);
            }
            int a = 0, b = 0, w = 0;
            while (a < au->n || b < av->n) {
                int32_t x;
                if (b >= av->n || (a < au->n && au->v[a] < av->v[b])) x = au->v[a++];
                else if (a >= au->n || av->v[b] < au->v[a]) x = av->v[b++];
                else { x = au->v[a]; a++; b++; }
                if (x != u && x != v) tmp[w++] = x;
            }
            if (w > au->cap) {
                au->cap = w;
                au->v = (int32_t*)realloc(au->v, sizeof(int32_t) * (size_t)w);
            }
            memcpy(au->v, tmp, sizeof(int32_t) * (size_t)w);
            au->n = w;
            if (hn + 1 >= hcap) {
                hcap *= 2;
                h = (hent*)realloc(h, sizeof(hent) * (size_t)hcap);
            }
            hent x = {w, u};
            hpush(h, &hn, x);
        }
        free(av->v);
        av->v = NULL;
        av->n = av->cap = 0;
    }
    free(tmp);
    free(done);
    free(h);
}

/* ------------------------------------------------------------------ symbolic factorisation (Sections 4.1, 4.3) */

/* Column structures of L by symbolic elimination in the order given by iperm (old->new):
 * struct(j) = {i > j : K_ij != 0} U  union over children c of struct(c) \ {j},
 * parent(j) = min struct(j).  Returns parent and the structures (new numbering). */
static void symbolic(int N, ivec* adj0, const int32_t* perm, const int32_t* iperm,
                     int32_t* parent, ivec* st) {
    ivec* kids = (ivec*)calloc((size_t)N, sizeof(ivec));
    char* mark = (char*)calloc((size_t)N, 1);
    for (int j = 0; j < N; ++j) {
        ivec s = {0, 0, 0};
        int old = perm[j];
        for (int t = 0; t < adj0[old].n; ++t) {
            int i = iperm[adj0[old].v[t]];
            if (i > j && !mark[i]) { mark[i] = 1; iv_push(&s, i); }
        }
        for (int t = 0; t < kids[j].n; ++t) {
            ivec* cs = &st[kids[j].v[t]];
            for (int q = 0; q < cs->n; ++q) {
                int i = cs->v[q];
                if (i != j && !mark[i]) { mark[i] = 1; iv_push(&s, i); }
            }
        }
        for (int q = 0; q < s.n; ++q) mark[s.v[q]] = 0;
        qsort(s.v, (size_t)s.n, sizeof(int32_t), cmp_i32);
        st[j] = s;
        parent[j] = s.n ? s.v[0] : -1;
        if (parent[j] >= 0) iv_push(&kids[parent[j]], j);
    }
    for (int j = 0; j < N; ++j) free(kids[j].v);
    free(kids);
    free(mark);
}

/* Postorder of a forest (children visited in ascending index, roots ascending). */
static void postorder(int N, const int32_t* parent, int32_t* post /* post[k] = node */) {
    int32_t* head = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    int32_t* next = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    int32_t* stack = (int32_t*)malloc(sizeof(int32_t) * (size_t)N);
    for (int j = 0; j < N; ++j) head[j] = -1;
    for (int j = N - 1; j >= 0; --j) /* insert in reverse so lists are ascending */
        if (parent[j] >= 0) { next[j] = head[parent[j]]; head[parent[j]] = j; }
    int k = 0;
    for (int r = 0; r < N; ++r) {
        if (parent[r] >= 0) continue;
        int top = 0;
        stack[top++] = r;
        while (top) {
            int v = stack[top - 1];
            int c = head[v];
            if (c >= 0) {
                head[v] = next[c];
                stack[top++] = c;
            } else {
                post[k++] = v;
                --top;
            }
        }
    }
    free(head); free(next); free(stack);
}

/* Lower pattern of K (diagonal + lower adjacency, original numbering) and a copy of A's
 * pattern: everything the value formation and the residual need, and no factorisation. */
static orc_sym* pattern_only(int m, int n, const int64_t* cp, const int32_t* ri, int mode,
                             const int64_t* qcp, const int32_t* qri, ivec** adj_out) {
    orc_sym* S = (orc_sym*)calloc(1, sizeof(orc_sym));
    S->m = m; S->n = n; S->mode = mode;
    int N;
    ivec* adj = build_adjacency(m, n, cp, ri, mode, qcp, qri, &N);
    if (qcp) {
        S->qcp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
        memcpy(S->qcp, qcp, sizeof(int64_t) * (size_t)(n + 1));
        S->qri = (int32_t*)malloc(sizeof(int32_t) * (size_t)(qcp[n] ? qcp[n] : 1));
        memcpy(S->qri, qri, sizeof(int32_t) * (size_t)qcp[n]);
    }
    S->N = N;
    S->acp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
    memcpy(S->acp, cp, sizeof(int64_t) * (size_t)(n + 1));
    S->ari = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cp[n] ? cp[n] : 1));
    memcpy(S->ari, ri, sizeof(int32_t) * (size_t)cp[n]);
    S->kp = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
    for (int v = 0; v < N; ++v) {
        int64_t c = 1;
        for (int t = 0; t < adj[v].n; ++t) c += adj[v].v[t] > v;
        S->kp[v + 1] = S->kp[v] + c;
    }
    S->ki = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->kp[N] ? S->kp[N] : 1));
    for (int v = 0; v < N; ++v) {
        int64_t w = S->kp[v];
        S->ki[w++] = v;
        for (int t = 0; t < adj[v].n; ++t)
            if (adj[v].v[t] > v) S->ki[w++] = adj[v].v[t];
    }
    if (adj_out) {
        *adj_out = adj;
    } else {
        for (int v = 0; v < N; ++v) free(adj[v].v);
        free(adj);
    }
    return S;
}

/* Q's lower triangle: rows >= the column, strictly increasing, inside [0, n) */
static int q_pattern_ok(int n, const int64_t* qcp, const int32_t* qri) {
    if (qcp[0] != 0) return 0;
    for (int j = 0; j < n; ++j) {
        if (qcp[j + 1] < qcp[j]) return 0;
        for (int64_t e = qcp[j]; e < qcp[j + 1]; ++e) {
            if (qri[e] < j || qri[e] >= n) return 0;
            if (e > qcp[j] && qri[e] <= qri[e - 1]) return 0;
        }
    }
    return 1;
}

static int analyse_impl(int m, int n, const int64_t* cp, const int32_t* ri, int mode,
                        const int64_t* qcp, const int32_t* qri, const int32_t* user_perm,
                        orc_sym** out);

int orc_analyse(int m, int n, const int64_t* cp, const int32_t* ri, int mode,
                const int32_t* user_perm, orc_sym** out) {
    return analyse_impl(m, n, cp, ri, mode, NULL, NULL, user_perm, out);
}

int orc_analyse_qp(int m, int n, const int64_t* cp, const int32_t* ri, const int64_t* qcp,
                   const int32_t* qri, const int32_t* user_perm, orc_sym** out) {
    if (n < 0 || !qcp || !qri || !q_pattern_ok(n, qcp, qri)) return -1;
    return analyse_impl(m, n, cp, ri, ORC_AS, qcp, qri, user_perm, out);
}

static int analyse_impl(int m, int n, const int64_t* cp, const int32_t* ri, int mode,
                        const int64_t* qcp, const int32_t* qri, const int32_t* user_perm,
                        orc_sym** out) {
    if (m < 0 || n < 0 || !cp || !ri || !out) return -1;
    ivec* adj = NULL;
    orc_sym* S = pattern_only(m, n, cp, ri, mode, qcp, qri, &adj);
    int N = S->N;
    /* ordering */
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    if (user_perm) {
        memcpy(order, user_perm, sizeof(int32_t) * (size_t)N);
    } else {
        ivec* work = (ivec*)calloc((size_t)N, sizeof(ivec));
        for (int v = 0; v < N; ++v) {
            work[v].n = work[v].cap = adj[v].n;
            work[v].v = (int32_t*)malloc(sizeof(int32_t) * (size_t)(adj[v].n ? adj[v].n : 1));
            memcpy(work[v].v, adj[v].v, sizeof(int32_t) * (size_t)adj[v].n);
        }
        min_degree(N, work, order);
        for (int v = 0; v < N; ++v) free(work[v].v);
        free(work);
    }
    int32_t* iorder = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    for (int k = 0; k < N; ++k) iorder[k] = -1;
    for (int k = 0; k < N; ++k) {
        if (order[k] < 0 || order[k] >= N || iorder[order[k]] >= 0) {
            for (int v = 0; v < N; ++v) free(adj[v].v);
            free(adj); free(order); free(iorder); orc_sym_free(S);
            return -2;
        }
        iorder[order[k]] = k;
    }
    /* etree in this order, then postorder it (Section 4.3) */
    int32_t* par0 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    ivec* st = (ivec*)calloc((size_t)N, sizeof(ivec));
    symbolic(N, adj, order, iorder, par0, st);
    for (int j = 0; j < N; ++j) free(st[j].v);
    int32_t* post = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    postorder(N, par0, post);
    S->perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    S->iperm = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    for (int k = 0; k < N; ++k) S->perm[k] = order[post[k]];
    for (int k = 0; k < N; ++k) S->iperm[S->perm[k]] = k;
    free(order); free(iorder); free(par0); free(post);
    /* structures in the final numbering */
    S->parent = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    memset(st, 0, sizeof(ivec) * (size_t)N);
    symbolic(N, adj, S->perm, S->iperm, S->parent, st);
    for (int v = 0; v < N; ++v) free(adj[v].v);
    free(adj);
    S->colcount = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N ? N : 1));
    S->nnzL = 0;
    S->flops = 0;
    for (int j = 0; j < N; ++j) {
        S->colcount[j] = st[j].n + 1;
        S->nnzL += st[j].n + 1;
        S->flops += (double)st[j].n * (st[j].n + 3);
    }
    /* fundamental supernodes (Section 4.1: consecutive columns with the same structure;
     * j+1 joins j when parent(j) = j+1, j is its only child, and the counts chain) */
    int32_t* nkids = (int32_t*)calloc((size_t)N + 1, sizeof(int32_t));
    for (int j = 0; j < N; ++j)
        if (S->parent[j] >= 0) nkids[S->parent[j]]++;
    S->snptr = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N + 1));
    S->col2sn = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    int ns = 0;
    for (int j = 0; j < N; ++j) {
        int join = j > 0 && S->parent[j - 1] == j && nkids[j] == 1 &&
                   S->colcount[j - 1] == S->colcount[j] + 1;
        if (!join) S->snptr[ns++] = j;
        S->col2sn[j] = ns - 1;
    }
    S->snptr[ns] = N;
    S->nsuper = ns;
    free(nkids);
    S->snparent = (int32_t*)malloc(sizeof(int32_t) * (size_t)(ns ? ns : 1));
    S->rowptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns + 1));
    S->rowptr[0] = 0;
    S->maxfront = 0;
    for (int s = 0; s < ns; ++s) {
        int c0 = S->snptr[s], c1 = S->snptr[s + 1];
        int64_t f = (c1 - c0) + st[c1 - 1].n;
        S->rowptr[s + 1] = S->rowptr[s] + f;
        if (f > S->maxfront) S->maxfront = f;
        int pl = S->parent[c1 - 1];
        S->snparent[s] = pl >= 0 ? S->col2sn[pl] : -1;
    }
    S->rows = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->rowptr[ns] ? S->rowptr[ns] : 1));
    for (int s = 0; s < ns; ++s) {
        int c0 = S->snptr[s], c1 = S->snptr[s + 1];
        int64_t w = S->rowptr[s];
        for (int c = c0; c < c1; ++c) S->rows[w++] = c;
        for (int t = 0; t < st[c1 - 1].n; ++t) S->rows[w++] = st[c1 - 1].v[t];
    }
    for (int j = 0; j < N; ++j) free(st[j].v);
    free(st);
    *out = S;
    return 0;
}

void orc_sym_free(orc_sym* S) {
    if (!S) return;
    free(S->kp); free(S->ki); free(S->perm); free(S->iperm); free(S->parent);
    free(S->colcount); free(S->snptr); free(S->snparent); free(S->col2sn);
    free(S->rowptr); free(S->rows); free(S->acp); free(S->ari); free(S->qcp); free(S->qri);
    free(S);
}

void orc_sym_info(const orc_sym* S, int64_t* info) {
    info[0] = S->N;
    info[1] = S->nsuper;
    info[2] = S->nnzL;
    info[3] = S->maxfront;
    info[4] = (int64_t)S->flops;
}
void orc_sym_perm(const orc_sym* S, int32_t* p) { memcpy(p, S->perm, sizeof(int32_t) * (size_t)S->N); }
void orc_sym_parent(const orc_sym* S, int32_t* p) { memcpy(p, S->parent, sizeof(int32_t) * (size_t)S->N); }
void orc_sym_colcount(const orc_sym* S, int64_t* c) { memcpy(c, S->colcount, sizeof(int64_t) * (size_t)S->N); }
void orc_sym_snptr(const orc_sym* S, int32_t* p) { memcpy(p, S->snptr, sizeof(int32_t) * (size_t)(S->nsuper + 1)); }
void orc_sym_snparent(const orc_sym* S, int32_t* p) { memcpy(p, S->snparent, sizeof(int32_t) * (size_t)S->nsuper); }
void orc_sym_front_rows(const orc_sym* S, int64_t* rp, int32_t* rows) {
    memcpy(rp, S->rowptr, sizeof(int64_t) * (size_t)(S->nsuper + 1));
    memcpy(rows, S->rows, sizeof(int32_t) * (size_t)S->rowptr[S->nsuper]);
}

/* ------------------------------------------------------------------ values of K (Sections 3, 3.2) */

/* Q_jj of a quadratic program (0 if absent or an LP) */
static double q_diag(const int64_t* qcp, const int32_t* qri, const double* qval, int j) {
    if (!qcp || qcp[j] == qcp[j + 1] || qri[qcp[j]] != j) return 0.0;
    return qval[qcp[j]];
}

/* K0 = the matrix before static shifts: AS: [[-diag(1/Theta), A^T],[A, 0]] (equation
 * (augsys)), for a quadratic program [[-(Q + diag(1/Theta)), A^T],[A, 0]]; NE:
 * A diag(theta~) A^T with theta~_j = 1/(1/Theta_j + rho) (equations (normeq),
 * (regul_matrix)), every entry summed over the columns j of A in ascending order.
 * Values are stored on S->kp/ki (lower part, original numbering). */
static double* form_k0(const orc_sym* S, const double* aval, const double* qval,
                       const double* theta, double rho) {
    int m = S->m, n = S->n, N = S->N;
    double* kval = (double*)calloc((size_t)(S->kp[N] ? S->kp[N] : 1), sizeof(double));
    if (S->mode == ORC_AS) {
        for (int j = 0; j < n; ++j) {
            /* diagonal of x_j; -rho is added at pivot time */
            kval[S->kp[j]] = -(1.0 / theta[j] + q_diag(S->qcp, S->qri, qval, j));
            /* the lower entries of column j in ascending rows: first the x rows k > j with
             * Q_kj != 0, then the y rows n+i with A_ij != 0 */
            int64_t w = S->kp[j] + 1;
            if (S->qcp)
                for (int64_t e = S->qcp[j]; e < S->qcp[j + 1]; ++e)
                    if (S->qri[e] != j) {
                        if (S->ki[w] != S->qri[e]) { free(kval); return NULL; }
                        kval[w++] = -qval[e];
                    }
            for (int64_t e = S->acp[j]; e < S->acp[j + 1]; ++e) {
                if (S->ki[w] != n + S->ari[e]) { free(kval); return NULL; }
                kval[w++] = aval[e];
            }
        }
        /* y diagonals are 0 */
    } else {
        /* CSR of A to walk the columns j of row k in ascending order */
        int64_t* rp = (int64_t*)calloc((size_t)m + 1, sizeof(int64_t));
        for (int64_t e = 0; e < S->acp[n]; ++e) rp[S->ari[e] + 1]++;
        for (int i = 0; i < m; ++i) rp[i + 1] += rp[i];
        int32_t* rc = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->acp[n] ? S->acp[n] : 1));
        double* rv = (double*)malloc(sizeof(double) * (size_t)(S->acp[n] ? S->acp[n] : 1));
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)m);
        memcpy(fill, rp, sizeof(int64_t) * (size_t)m);
        for (int j = 0; j < n; ++j)
            for (int64_t e = S->acp[j]; e < S->acp[j + 1]; ++e) {
                int i = S->ari[e];
                rc[fill[i]] = j;
                rv[fill[i]++] = aval[e];
            }
        double* tt = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
        for (int j = 0; j < n; ++j) tt[j] = 1.0 / (1.0 / theta[j] + rho);
        double* acc = (double*)calloc((size_t)m, sizeof(double));
        for (int k = 0; k < m; ++k) {
            /* column k of the lower part: K_ik = sum_j A_ij tt_j A_kj, i >= k */
            for (int64_t q = rp[k]; q < rp[k + 1]; ++q) {
                int j = rc[q];
                double akj = rv[q];
                for (int64_t e = S->acp[j]; e < S->acp[j + 1]; ++e) {
                    int i = S->ari[e];
                    if (i >= k) acc[i] += (aval[e] * tt[j]) * akj;
                }
            }
            for (int64_t e = S->kp[k]; e < S->kp[k + 1]; ++e) {
                kval[e] = acc[S->ki[e]];
                acc[S->ki[e]] = 0.0;
            }
        }
        free(acc); free(tt); free(fill); free(rv); free(rc); free(rp);
    }
    return kval;
}

/* ||K_static||_1 = max column sum of |K0 + diag(static shifts)| (symmetric, = inf-norm). */
static double knorm_of(const orc_sym* S, const double* kval, double rho, double delta,
                       double* rowsum /* may be NULL, length N */) {
    int N = S->N;
    double* cs = (double*)calloc((size_t)(N ? N : 1), sizeof(double));
    for (int c = 0; c < N; ++c)
        for (int64_t e = S->kp[c]; e < S->kp[c + 1]; ++e) {
            int r = S->ki[e];
            double v = kval[e];
            if (r == c) {
                double s = (S->mode == ORC_AS && c < S->n) ? -rho : delta;
                cs[c] += fabs(v + s);
            } else {
                cs[c] += fabs(v);
                cs[r] += fabs(v);
            }
        }
    double mx = 0;
    for (int c = 0; c < N; ++c) if (cs[c] > mx) mx = cs[c];
    if (rowsum) memcpy(rowsum, cs, sizeof(double) * (size_t)N);
    free(cs);
    return mx;
}

/* ------------------------------------------------------------------ dense front (Sections 4.4-4.6) */

#define FE(F, f, i, j) (F)[(size_t)(i) + (size_t)(j) * (size_t)(f)]

/* symmetric interchange of positions a and b: rows and columns of the whole front */
static void sym_swap(double* F, int f, int a, int b, int8_t* sigma, double* shift, int32_t* perm) {
    if (a == b) return;
    for (int j = 0; j < f; ++j) { double t = FE(F, f, a, j); FE(F, f, a, j) = FE(F, f, b, j); FE(F, f, b, j) = t; }
    for (int i = 0; i < f; ++i) { double t = FE(F, f, i, a); FE(F, f, i, a) = FE(F, f, i, b); FE(F, f, i, b) = t; }
    int8_t ts = sigma[a]; sigma[a] = sigma[b]; sigma[b] = ts;
    double tz = shift[a]; shift[a] = shift[b]; shift[b] = tz;
    int32_t tp = perm[a]; perm[a] = perm[b]; perm[b] = tp;
}

static void front_factor(int f, int p, double* F, int8_t* sigma, double* shift, int32_t* perm,
                         double knorm, const orc_opts* o, double* d, double* doff, int8_t* ptype,
                         double* edyn, int8_t* eflag, orc_stats* st) {
    const double alpha = o->alpha;
    const double tiny = o->eps_lift * knorm; /* delta * ||M||_1 of Section 4.5 */
    for (int k = 0; k < f; ++k) perm[k] = k;
    for (int ws = 0; ws < p; ws += o->nb) {
        int we = ws + o->nb < p ? ws + o->nb : p; /* window = diagonal block B_D */
        int k = ws;
        while (k < we) {
            /* presort: largest |diagonal| of the window to position k (Section 4.5) */
            if (o->presort) {
                int q = k;
                for (int j = k + 1; j < we; ++j)
                    if (fabs(FE(F, f, j, j)) > fabs(FE(F, f, q, q))) q = j;
                sym_swap(F, f, k, q, sigma, shift, perm);
            }
            /* Bunch-Kaufman variant (Section 4.5); tests read only window rows */
            double gp = 0.0;
            int r = -1;
            for (int i = k + 1; i < we; ++i)
                if (fabs(FE(F, f, i, k)) > gp) { gp = fabs(FE(F, f, i, k)); r = i; }
            double akk = fabs(FE(F, f, k, k));
            int two = 0, lifted = 0;
            double fkk_before = FE(F, f, k, k);
            if ((akk > gp ? akk : gp) <= tiny) {
                FE(F, f, k, k) = sigma[k] * tiny; /* lift */
                lifted = 1;
            } else if (akk >= alpha * gp) {
                /* 1x1 at k */
            } else {
                double gr = 0.0;
                for (int i = k; i < we; ++i)
                    if (i != r && fabs(FE(F, f, i, r)) > gr) gr = fabs(FE(F, f, i, r));
                if (akk * gr >= alpha * gp * gp) {
                    /* 1x1 at k */
                } else if (fabs(FE(F, f, r, r)) >= alpha * gr) {
                    sym_swap(F, f, k, r, sigma, shift, perm);
                    fkk_before = FE(F, f, k, k);
                    st->nbkd++;
                } else {
                    sym_swap(F, f, k + 1, r, sigma, shift, perm);
                    two = 1;
                }
            }
            if (two) {
                double a = FE(F, f, k, k) + shift[k];
                double b = FE(F, f, k + 1, k);
                double c = FE(F, f, k + 1, k + 1) + shift[k + 1];
                double det = a * c - b * b;
                if (det == 0.0) { /* fall back to a lifted 1x1 pivot at k */
                    two = 0;
                    fkk_before = FE(F, f, k, k);
                    FE(F, f, k, k) = sigma[k] * tiny;
                    lifted = 1;
                } else {
                    /* 2x2 pivot: L2 = F[k+2:, k:k+2] D2^{-1}; Schur update */
                    d[k] = a; d[k + 1] = c; doff[k] = b; doff[k + 1] = 0.0;
                    ptype[k] = 1; ptype[k + 1] = 2;
                    if (eflag) eflag[k] = eflag[k + 1] = 0;
                    edyn[k] = 0.0; edyn[k + 1] = 0.0;
                    for (int j = k + 2; j < f; ++j) {
                        double u0 = FE(F, f, j, k), u1 = FE(F, f, j, k + 1);
                        double l0 = (u0 * c - u1 * b) / det;
                        double l1 = (u1 * a - u0 * b) / det;
                        for (int i = k + 2; i < f; ++i)
                            FE(F, f, i, j) -= FE(F, f, i, k) * l0 + FE(F, f, i, k + 1) * l1;
                    }
                    for (int i = k + 2; i < f; ++i) {
                        double u0 = FE(F, f, i, k), u1 = FE(F, f, i, k + 1);
                        FE(F, f, i, k) = (u0 * c - u1 * b) / det;
                        FE(F, f, i, k + 1) = (u1 * a - u0 * b) / det;
                    }
                    FE(F, f, k + 1, k) = 0.0;
                    st->n2x2++;
                    if (det < 0) { st->nneg++; st->npos++; }
                    else if (a + c > 0) st->npos += 2;
                    else st->nneg += 2;
                    k += 2;
                    continue;
                }
            }
            /* 1x1 pivot at k */
            if (lifted) st->nlift++;
            double dk = FE(F, f, k, k) + shift[k]; /* static regularisation after the pivot */
            /* Proposition 3 against the window's same-sign columns (Section 4.6) */
            double beta = 0.0;
            for (int j = k + 1; j < we; ++j) {
                if (sigma[j] != sigma[k]) continue;
                double den = fabs(FE(F, f, j, j) + shift[j]);
                if (den == 0.0) { st->nzskip++; continue; }
                double q = FE(F, f, j, k) * FE(F, f, j, k) / den;
                if (q > beta) beta = q;
            }
            int8_t ef = lifted ? ORC_EF_LIFT : 0;
            if (fabs(dk) < beta) { dk = sigma[k] * beta; st->nprop3++; ef |= ORC_EF_PROP3; }
            if (!((sigma[k] > 0 && dk > 0) || (sigma[k] < 0 && dk < 0))) {
                double mag = fabs(dk);
                if (beta > mag) mag = beta;
                if (tiny > mag) mag = tiny;
                dk = sigma[k] * mag;
                st->nsign++;
                ef |= ORC_EF_SIGN;
            }
            if (eflag) eflag[k] = ef;
            d[k] = dk; doff[k] = 0.0; ptype[k] = 0;
            edyn[k] = dk - (fkk_before + shift[k]);
            if (fabs(edyn[k]) > st->max_edyn) st->max_edyn = fabs(edyn[k]);
            if (fabs(edyn[k]) > o->tau_big * knorm) st->large_reg = 1;
            if (dk > 0) st->npos++; else if (dk < 0) st->nneg++; else st->nzero++;
            /* eliminate over all remaining rows of the front (right-looking) */
            for (int j = k + 1; j < f; ++j) {
                double wj = FE(F, f, j, k);
                for (int i = k + 1; i < f; ++i) FE(F, f, i, j) -= (FE(F, f, i, k) / dk) * wj;
            }
            for (int i = k + 1; i < f; ++i) FE(F, f, i, k) /= dk;
            k += 1;
        }
    }
}

void orc_front_factor(int f, int p, double* F, int8_t* sigma, double* shift, int32_t* perm,
                      double knorm, const orc_opts* o, double* d, double* doff, int8_t* ptype,
                      double* edyn, orc_stats* st) {
    front_factor(f, p, F, sigma, shift, perm, knorm, o, d, doff, ptype, edyn, NULL, st);
}

/* ------------------------------------------------------------------ multifrontal factorisation (Section 4.1) */

int orc_factorise(const orc_sym* S, const double* aval, const double* theta, double rho,
                  double delta, const orc_opts* o, orc_num** out) {
    if (S->qcp) return -1; /* a quadratic program needs Q's values */
    return orc_factorise_qp(S, aval, NULL, theta, rho, delta, o, out);
}

int orc_factorise_qp(const orc_sym* S, const double* aval, const double* qval, const double* theta,
                     double rho, double delta, const orc_opts* o, orc_num** out) {
    int N = S->N, n = S->n;
    if (S->qcp && !qval) return -1;
    for (int j = 0; j < n; ++j)
        if (!(theta[j] > 0) || !isfinite(theta[j])) return -1;
    orc_num* R = (orc_num*)calloc(1, sizeof(orc_num));
    R->S = S;
    R->opts = *o;
    R->rho = rho;
    R->delta = delta;
    R->theta = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
    memcpy(R->theta, theta, sizeof(double) * (size_t)n);
    int64_t annz = S->acp[n];
    R->aval = (double*)malloc(sizeof(double) * (size_t)(annz ? annz : 1));
    memcpy(R->aval, aval, sizeof(double) * (size_t)annz);
    if (S->qcp) {
        int64_t qnnz = S->qcp[n];
        R->qval = (double*)malloc(sizeof(double) * (size_t)(qnnz ? qnnz : 1));
        memcpy(R->qval, qval, sizeof(double) * (size_t)qnnz);
    }
    R->kval = form_k0(S, aval, R->qval, theta, rho);
    if (!R->kval) { orc_num_free(R); return -3; }
    R->knorm = knorm_of(S, R->kval, rho, delta, NULL);
    int ns = S->nsuper;
    R->Lptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(ns + 1));
    R->Lptr[0] = 0;
    for (int s = 0; s < ns; ++s) {
        int64_t f = S->rowptr[s + 1] - S->rowptr[s];
        int64_t p = S->snptr[s + 1] - S->snptr[s];
        R->Lptr[s + 1] = R->Lptr[s] + f * p;
    }
    R->L = (double*)calloc((size_t)(R->Lptr[ns] ? R->Lptr[ns] : 1), sizeof(double));
    R->d = (double*)calloc((size_t)(N ? N : 1), sizeof(double));
    R->doff = (double*)calloc((size_t)(N ? N : 1), sizeof(double));
    R->ptype = (int8_t*)calloc((size_t)(N ? N : 1), 1);
    R->edyn = (double*)calloc((size_t)(N ? N : 1), sizeof(double));
    R->eflag = (int8_t*)calloc((size_t)(N ? N : 1), 1);
    R->lperm = (int32_t*)calloc((size_t)(N ? N : 1), sizeof(int32_t));
    /* K0 lower entries regrouped by final column (new numbering) */
    int64_t knnz = S->kp[N];
    int64_t* cp2 = (int64_t*)calloc((size_t)N + 1, sizeof(int64_t));
    for (int c = 0; c < N; ++c)
        for (int64_t e = S->kp[c]; e < S->kp[c + 1]; ++e) {
            int a = S->iperm[S->ki[e]], b = S->iperm[c];
            cp2[(a < b ? a : b) + 1]++;
        }
    for (int c = 0; c < N; ++c) cp2[c + 1] += cp2[c];
    int32_t* r2 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(knnz ? knnz : 1));
    double* v2 = (double*)malloc(sizeof(double) * (size_t)(knnz ? knnz : 1));
    int64_t* fl = (int64_t*)malloc(sizeof(int64_t) * (size_t)(N ? N : 1));
    memcpy(fl, cp2, sizeof(int64_t) * (size_t)N);
    for (int c = 0; c < N; ++c)
        for (int64_t e = S->kp[c]; e < S->kp[c + 1]; ++e) {
            int a = S->iperm[S->ki[e]], b = S->iperm[c];
            int lo = a < b ? a : b, hi = a < b ? b : a;
            r2[fl[lo]] = hi;
            v2[fl[lo]++] = R->kval[e];
        }
    free(fl);
    /* children lists (ascending) and CB storage */
    double** cb = (double**)calloc((size_t)(ns ? ns : 1), sizeof(double*));
    int32_t* map = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    for (int i = 0; i < N; ++i) map[i] = -1;
    for (int s = 0; s < ns; ++s) {
        int c0 = S->snptr[s], p = S->snptr[s + 1] - c0;
        int f = (int)(S->rowptr[s + 1] - S->rowptr[s]);
        const int32_t* R_s = S->rows + S->rowptr[s];
        for (int a = 0; a < f; ++a) map[R_s[a]] = a;
        double* Fr = (double*)calloc((size_t)f * (size_t)f, sizeof(double));
        /* original entries of the pivot columns */
        for (int c = c0; c < c0 + p; ++c)
            for (int64_t e = cp2[c]; e < cp2[c + 1]; ++e) {
                int a = map[r2[e]], b = map[c];
                FE(Fr, f, a, b) += v2[e];
                if (a != b) FE(Fr, f, b, a) += v2[e];
            }
        /* children contribution blocks, children in ascending order (Section 4.3) */
        for (int t = 0; t < s; ++t) {
            if (S->snparent[t] != s) continue;
            int tp = S->snptr[t + 1] - S->snptr[t];
            int tf = (int)(S->rowptr[t + 1] - S->rowptr[t]);
            int tc = tf - tp;
            const int32_t* R_t = S->rows + S->rowptr[t] + tp;
            for (int b = 0; b < tc; ++b)
                for (int a = 0; a < tc; ++a)
                    FE(Fr, f, map[R_t[a]], map[R_t[b]]) += cb[t][(size_t)a + (size_t)b * tc];
            free(cb[t]);
            cb[t] = NULL;
        }
        /* expected signs and static shifts per row (Section 4.5) */
        int8_t* sg = (int8_t*)malloc((size_t)f);
        double* sh = (double*)malloc(sizeof(double) * (size_t)f);
        int32_t* pm = (int32_t*)malloc(sizeof(int32_t) * (size_t)f);
        for (int a = 0; a < f; ++a) {
            int old = S->perm[R_s[a]];
            int primal = (S->mode == ORC_AS) && old < n;
            sg[a] = primal ? -1 : 1;
            sh[a] = primal ? -rho : delta;
        }
        front_factor(f, p, Fr, sg, sh, pm, R->knorm, o, R->d + c0, R->doff + c0, R->ptype + c0,
                     R->edyn + c0, R->eflag + c0, &R->st);
        for (int k = 0; k < p; ++k) R->lperm[c0 + k] = pm[k];
        double* Ls = R->L + R->Lptr[s];
        for (int k = 0; k < p; ++k)
            for (int a = 0; a < f; ++a) Ls[(size_t)a + (size_t)k * f] = a > k ? FE(Fr, f, a, k) : (a == k ? 1.0 : 0.0);
        int c = f - p;
        if (c > 0) {
            cb[s] = (double*)malloc(sizeof(double) * (size_t)c * (size_t)c);
            for (int b = 0; b < c; ++b)
                for (int a = 0; a < c; ++a) cb[s][(size_t)a + (size_t)b * c] = FE(Fr, f, p + a, p + b);
        }
        for (int a = 0; a < f; ++a) map[R_s[a]] = -1;
        free(Fr); free(sg); free(sh); free(pm);
    }
    for (int s = 0; s < ns; ++s) free(cb[s]);
    free(cb); free(map); free(cp2); free(r2); free(v2);
    *out = R;
    return 0;
}

void orc_num_free(orc_num* R) {
    if (!R) return;
    free(R->theta); free(R->aval); free(R->qval); free(R->kval); free(R->Lptr); free(R->L); free(R->d);
    free(R->doff); free(R->ptype); free(R->edyn); free(R->eflag); free(R->lperm);
    free(R);
}

void orc_num_stats(const orc_num* R, orc_stats* st) { *st = R->st; }
void orc_num_eflags(const orc_num* R, int8_t* eflag) {
    memcpy(eflag, R->eflag, (size_t)R->S->N);
}
double orc_num_knorm(const orc_num* R) { return R->knorm; }

/* index (new numbering) of front row a of supernode s after pivoting */
static int row_index(const orc_sym* S, const orc_num* R, int s, int a) {
    int c0 = S->snptr[s], p = S->snptr[s + 1] - c0;
    return a < p ? c0 + R->lperm[c0 + a] : S->rows[S->rowptr[s] + a];
}

void orc_num_export(const orc_num* R, int32_t* fperm, double* Ld, double* d, double* doff,
                    int8_t* ptype, double* edyn) {
    const orc_sym* S = R->S;
    int N = S->N;
    int32_t* pos = (int32_t*)malloc(sizeof(int32_t) * (size_t)(N ? N : 1));
    for (int s = 0; s < S->nsuper; ++s)
        for (int k = S->snptr[s]; k < S->snptr[s + 1]; ++k)
            pos[S->snptr[s] + R->lperm[k]] = k;
    for (int k = 0; k < N; ++k) fperm[k] = S->perm[S->snptr[S->col2sn[k]] + R->lperm[k]];
    if (Ld) {
        memset(Ld, 0, sizeof(double) * (size_t)N * (size_t)N);
        for (int s = 0; s < S->nsuper; ++s) {
            int c0 = S->snptr[s], p = S->snptr[s + 1] - c0;
            int f = (int)(S->rowptr[s + 1] - S->rowptr[s]);
            const double* Ls = R->L + R->Lptr[s];
            for (int k = 0; k < p; ++k)
                for (int a = k; a < f; ++a)
                    Ld[(size_t)pos[row_index(S, R, s, a)] + (size_t)(c0 + k) * N] = Ls[(size_t)a + (size_t)k * f];
        }
    }
    memcpy(d, R->d, sizeof(double) * (size_t)N);
    memcpy(doff, R->doff, sizeof(double) * (size_t)N);
    memcpy(ptype, R->ptype, (size_t)N);
    memcpy(edyn, R->edyn, sizeof(double) * (size_t)N);
    free(pos);
}

/* ------------------------------------------------------------------ solve (Section 4: forward, D, backward) */

/* Solve (L D L^T) w = w in place, w indexed in the new numbering. */
static void ldlt_solve(const orc_sym* S, const orc_num* R, double* w) {
    int ns = S->nsuper;
    for (int s = 0; s < ns; ++s) { /* forward with unit L, supernodes in postorder */
        int c0 = S->snptr[s], p = S->snptr[s + 1] - c0;
        int f = (int)(S->rowptr[s + 1] - S->rowptr[s]);
        const double* Ls = R->L + R->Lptr[s];
        for (int k = 0; k < p;) {
            if (R->ptype[c0 + k] == 1) {
                double z0 = w[row_index(S, R, s, k)], z1 = w[row_index(S, R, s, k + 1)];
                for (int a = k + 2; a < f; ++a)
                    w[row_index(S, R, s, a)] -= Ls[a + (size_t)k * f] * z0 + Ls[a + (size_t)(k + 1) * f] * z1;
                k += 2;
            } else {
                double z = w[row_index(S, R, s, k)];
                for (int a = k + 1; a < f; ++a) w[row_index(S, R, s, a)] -= Ls[a + (size_t)k * f] * z;
                k += 1;
            }
        }
    }
    for (int s = 0; s < ns; ++s) { /* block-diagonal D */
        int c0 = S->snptr[s], p = S->snptr[s + 1] - c0;
        for (int k = 0; k < p;) {
            if (R->ptype[c0 + k] == 1) {
                int i0 = row_index(S, R, s, k), i1 = row_index(S, R, s, k + 1);
                double a = R->d[c0 + k], b = R->doff[c0 + k], c = R->d[c0 + k + 1];
                double det = a * c - b * b;
                double u0 = w[i0], u1 = w[i1];
                w[i0] = (c * u0 - b * u1) / det;
                w[i1] = (a * u1 - b * u0) / det;
                k += 2;
            } else {
                w[row_index(S, R, s, k)] /= R->d[c0 + k];
                k += 1;
            }
        }
    }
    for (int s = ns - 1; s >= 0; --s) { /* backward with L^T, reverse postorder */
        int c0 = S->snptr[s], p = S->snptr[s + 1] - c0;
        int f = (int)(S->rowptr[s + 1] - S->rowptr[s]);
        const double* Ls = R->L + R->Lptr[s];
        for (int k = p - 1; k >= 0;) {
            if (R->ptype[c0 + k] == 2) {
                int k0 = k - 1;
                double s0 = 0, s1 = 0;
                for (int a = k0 + 2; a < f; ++a) {
                    double x = w[row_index(S, R, s, a)];
                    s0 += Ls[a + (size_t)k0 * f] * x;
                    s1 += Ls[a + (size_t)(k0 + 1) * f] * x;
                }
                w[row_index(S, R, s, k0)] -= s0;
                w[row_index(S, R, s, k0 + 1)] -= s1;
                k -= 2;
            } else {
                double s0 = 0;
                for (int a = k + 1; a < f; ++a) s0 += Ls[a + (size_t)k * f] * w[row_index(S, R, s, a)];
                w[row_index(S, R, s, k)] -= s0;
                k -= 1;
            }
        }
    }
}

/* ------------------------------------------------------------------ residual and backward error (Section 4.5) */

typedef struct {
    int m, n, mode, N;
    const int64_t* cp;
    const int32_t* ri;
    const double* av;
    const double* theta;
    double rho, delta;
    /* AS quadratic programs: Q's lower triangle, NULL for an LP */
    const int64_t* qcp;
    const int32_t* qri;
    const double* qv;
    /* NE: explicit K0 lower (original numbering) */
    const int64_t* kp;
    const int32_t* ki;
    const double* kv;
} sysdesc;

/* y = K_static x and ay = |K_static| |x| */
static void apply_k(const sysdesc* D, const double* x, double* y, double* ay) {
    int N = D->N;
    for (int i = 0; i < N; ++i) { y[i] = 0; ay[i] = 0; }
    if (D->mode == ORC_AS) {
        int n = D->n;
        for (int j = 0; j < n; ++j) {
            double dj = -(1.0 / D->theta[j] + q_diag(D->qcp, D->qri, D->qv, j) + D->rho);
            y[j] += dj * x[j];
            ay[j] += fabs(dj) * fabs(x[j]);
            if (D->qcp) /* off-diagonal -Q_kj, both triangles */
                for (int64_t e = D->qcp[j]; e < D->qcp[j + 1]; ++e) {
                    int k = D->qri[e];
                    if (k == j) continue;
                    double q = -D->qv[e];
                    y[j] += q * x[k];
                    ay[j] += fabs(q) * fabs(x[k]);
                    y[k] += q * x[j];
                    ay[k] += fabs(q) * fabs(x[j]);
                }
            for (int64_t e = D->cp[j]; e < D->cp[j + 1]; ++e) {
                int i = n + D->ri[e];
                double a = D->av[e];
                y[j] += a * x[i];
                ay[j] += fabs(a) * fabs(x[i]);
                y[i] += a * x[j];
                ay[i] += fabs(a) * fabs(x[j]);
            }
        }
        for (int i = 0; i < D->m; ++i) {
            y[n + i] += D->delta * x[n + i];
            ay[n + i] += D->delta * fabs(x[n + i]);
        }
    } else {
        for (int c = 0; c < N; ++c)
            for (int64_t e = D->kp[c]; e < D->kp[c + 1]; ++e) {
                int r = D->ki[e];
                double v = D->kv[e];
                if (r == c) v += D->delta;
                y[r] += v * x[c];
                ay[r] += fabs(v) * fabs(x[c]);
                if (r != c) {
                    y[c] += v * x[r];
                    ay[c] += fabs(v) * fabs(x[r]);
                }
            }
    }
}

static void backward_error(const sysdesc* D, double knorm, const double* rowsum,
                           const double* x, const double* b, double* r, double* nw, double* cw) {
    int N = D->N;
    double* kx = (double*)malloc(sizeof(double) * (size_t)(N ? N : 1));
    double* akx = (double*)malloc(sizeof(double) * (size_t)(N ? N : 1));
    apply_k(D, x, kx, akx);
    double rmax = 0, xmax = 0, bmax = 0, cmax = 0;
    for (int i = 0; i < N; ++i) {
        if (fabs(x[i]) > xmax) xmax = fabs(x[i]);
        if (fabs(b[i]) > bmax) bmax = fabs(b[i]);
    }
    const double u = 1.1102230246251565e-16;
    for (int i = 0; i < N; ++i) {
        double ri = b[i] - kx[i];
        if (r) r[i] = ri;
        if (fabs(ri) > rmax) rmax = fabs(ri);
        /* componentwise error with the small-denominator substitution of Arioli, Demmel
         * and Duff: (|K||x|)_i + ||x||_inf (|K| e)_i when the denominator is tiny */
        double den = akx[i] + fabs(b[i]);
        if (den <= 1000.0 * N * u * (rowsum[i] * xmax + fabs(b[i]))) den = akx[i] + xmax * rowsum[i];
        double c = den > 0 ? fabs(ri) / den : (ri == 0 ? 0 : INFINITY);
        if (c > cmax) cmax = c;
    }
    double den = knorm * xmax + bmax;
    *nw = den > 0 ? rmax / den : (rmax == 0 ? 0 : INFINITY);
    *cw = cmax;
    free(kx); free(akx);
}

/* explicit K0 for NE on a pattern built here (independent of any analyse) */
static void ne_explicit(int m, int n, const int64_t* cp, const int32_t* ri, const double* av,
                        const double* theta, double rho, int64_t** kpo, int32_t** kio,
                        double** kvo) {
    orc_sym* S = pattern_only(m, n, cp, ri, ORC_NE, NULL, NULL, NULL);
    double* kv = form_k0(S, av, NULL, theta, rho);
    *kpo = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m + 1));
    memcpy(*kpo, S->kp, sizeof(int64_t) * (size_t)(m + 1));
    *kio = (int32_t*)malloc(sizeof(int32_t) * (size_t)(S->kp[m] ? S->kp[m] : 1));
    memcpy(*kio, S->ki, sizeof(int32_t) * (size_t)S->kp[m]);
    *kvo = kv;
    orc_sym_free(S);
}

int orc_residual(int m, int n, const int64_t* cp, const int32_t* ri, const double* av,
                 int mode, const double* theta, double rho, double delta, const double* x,
                 const double* b, double* r, double* berr_nw, double* berr_cw, double* knorm) {
    return orc_residual_qp(m, n, cp, ri, av, mode, NULL, NULL, NULL, theta, rho, delta, x, b, r,
                           berr_nw, berr_cw, knorm);
}

int orc_residual_qp(int m, int n, const int64_t* cp, const int32_t* ri, const double* av,
                    int mode, const int64_t* qcp, const int32_t* qri, const double* qv,
                    const double* theta, double rho, double delta, const double* x,
                    const double* b, double* r, double* berr_nw, double* berr_cw, double* knorm) {
    if (qcp && (mode != ORC_AS || !qri || !qv || !q_pattern_ok(n, qcp, qri))) return -1;
    sysdesc D = {m, n, mode, mode == ORC_AS ? n + m : m, cp, ri, av, theta, rho, delta,
                 qcp, qri, qv, 0, 0, 0};
    int64_t* kp = NULL;
    int32_t* ki = NULL;
    double* kv = NULL;
    int N = D.N;
    double* rs = (double*)calloc((size_t)(N ? N : 1), sizeof(double));
    double kn = 0;
    if (mode == ORC_NE) {
        ne_explicit(m, n, cp, ri, av, theta, rho, &kp, &ki, &kv);
        D.kp = kp; D.ki = ki; D.kv = kv;
        for (int c = 0; c < N; ++c)
            for (int64_t e = kp[c]; e < kp[c + 1]; ++e) {
                int rr = ki[e];
                if (rr == c) rs[c] += fabs(kv[e] + delta);
                else { rs[c] += fabs(kv[e]); rs[rr] += fabs(kv[e]); }
            }
    } else {
        for (int j = 0; j < n; ++j) {
            rs[j] += fabs(1.0 / theta[j] + q_diag(qcp, qri, qv, j) + rho);
            if (qcp)
                for (int64_t e = qcp[j]; e < qcp[j + 1]; ++e)
                    if (qri[e] != j) {
                        rs[j] += fabs(qv[e]);
                        rs[qri[e]] += fabs(qv[e]);
                    }
            for (int64_t e = cp[j]; e < cp[j + 1]; ++e) {
                rs[j] += fabs(av[e]);
                rs[n + ri[e]] += fabs(av[e]);
            }
        }
        for (int i = 0; i < m; ++i) rs[n + i] += delta;
    }
    for (int i = 0; i < N; ++i) if (rs[i] > kn) kn = rs[i];
    backward_error(&D, kn, rs, x, b, r, berr_nw, berr_cw);
    if (knorm) *knorm = kn;
    free(kp); free(ki); free(kv); free(rs);
    return 0;
}

int orc_solve(const orc_sym* S, const orc_num* R, int nrhs, const double* r7, const double* r1,
              double* dx, double* dy, double* berr_nw, double* berr_cw, int* steps) {
    int m = S->m, n = S->n, N = S->N;
    const orc_opts* o = &R->opts;
    sysdesc D = {m, n, S->mode, N, S->acp, S->ari, R->aval, R->theta, R->rho, R->delta,
                 S->qcp, S->qri, R->qval, S->kp, S->ki, R->kval};
    double* rs = (double*)calloc((size_t)(N ? N : 1), sizeof(double));
    double kn = knorm_of(S, R->kval, R->rho, R->delta, rs);
    double* tt = (double*)malloc(sizeof(double) * (size_t)(n ? n : 1));
    for (int j = 0; j < n; ++j) tt[j] = 1.0 / (1.0 / R->theta[j] + R->rho);
    double* b = (double*)malloc(sizeof(double) * (size_t)(N ? N : 1));
    double* x = (double*)malloc(sizeof(double) * (size_t)(N ? N : 1));
    double* xb = (double*)malloc(sizeof(double) * (size_t)(N ? N : 1));
    double* r = (double*)malloc(sizeof(double) * (size_t)(N ? N : 1));
    double* w = (double*)malloc(sizeof(double) * (size_t)(N ? N : 1));
    for (int c = 0; c < nrhs; ++c) {
        const double* r7c = r7 ? r7 + (size_t)c * n : NULL;
        const double* r1c = r1 + (size_t)c * m;
        /* right-hand side of the system being factorised (equations (augsys), (normeq)) */
        if (S->mode == ORC_AS) {
            for (int j = 0; j < n; ++j) b[j] = r7c ? r7c[j] : 0.0;
            for (int i = 0; i < m; ++i) b[n + i] = r1c[i];
        } else {
            for (int i = 0; i < m; ++i) b[i] = r1c[i];
            if (r7c)
                for (int j = 0; j < n; ++j) /* r8 = r1 + A theta~ r7 */
                    for (int64_t e = S->acp[j]; e < S->acp[j + 1]; ++e)
                        b[S->ari[e]] += R->aval[e] * (tt[j] * r7c[j]);
        }
        /* x = (LDL^T)^{-1} b, then iterative refinement (Section 4.5) */
        for (int i = 0; i < N; ++i) w[S->iperm[i]] = b[i];
        ldlt_solve(S, R, w);
        for (int i = 0; i < N; ++i) x[i] = w[S->iperm[i]];
        double nw, cw;
        backward_error(&D, kn, rs, x, b, r, &nw, &cw);
        int st = 0;
        while (nw > o->target_berr && st < o->max_refine) {
            memcpy(xb, x, sizeof(double) * (size_t)N);
            for (int i = 0; i < N; ++i) w[S->iperm[i]] = r[i];
            ldlt_solve(S, R, w);
            for (int i = 0; i < N; ++i) x[i] += w[S->iperm[i]];
            double nw2, cw2;
            backward_error(&D, kn, rs, x, b, r, &nw2, &cw2);
            ++st;
            if (!(nw2 < nw)) { /* no improvement: keep the previous iterate */
                memcpy(x, xb, sizeof(double) * (size_t)N);
                backward_error(&D, kn, rs, x, b, r, &nw, &cw);
                break;
            }
            int stagnating = nw2 > 0.5 * nw;
            nw = nw2; cw = cw2;
            if (stagnating) break;
        }
        if (berr_nw) berr_nw[c] = nw;
        if (berr_cw) berr_cw[c] = cw;
        if (steps) steps[c] = st;
        if (S->mode == ORC_AS) {
            for (int j = 0; j < n; ++j) dx[(size_t)c * n + j] = x[j];
            for (int i = 0; i < m; ++i) dy[(size_t)c * m + i] = x[n + i];
        } else {
            for (int i = 0; i < m; ++i) dy[(size_t)c * m + i] = x[i];
            /* dx = theta~ (A^T dy - r7) */
            for (int j = 0; j < n; ++j) {
                double s = 0;
                for (int64_t e = S->acp[j]; e < S->acp[j + 1]; ++e) s += R->aval[e] * x[S->ari[e]];
                dx[(size_t)c * n + j] = tt[j] * (s - (r7c ? r7c[j] : 0.0));
            }
        }
    }
    free(rs); free(tt); free(b); free(x); free(xb); free(r); free(w);
    return 0;
}
