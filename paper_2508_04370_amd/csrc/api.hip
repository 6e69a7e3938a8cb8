// C ABI of the library: handles, analyse/upload, factorise and solve enqueueing, statistics,
// export and HIP graph capture.  Every numerical step runs in the kernels of kernels.hip.
#include <hip/hip_runtime.h>

#include <chrono>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/qdmf.h"
#include "device.hpp"
#include "plan.hpp"

using namespace qdmf;

struct qdmf_ctx {
    int device = 0;
    bool host_only = false;
    hipStream_t stream = nullptr;
    // lookahead: the second stream of the factorisation and the two events that order it
    // against the first (created by the analyse of a plan that uses them)
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_win = nullptr, ev_s2 = nullptr;
    qdmf_options opt{};
    std::string msg;

    Plan P;
    bool analysed = false, have_matrix = false, factorised = false;
    bool have_hessian = false;  // quadratic programs: qdmf_set_hessian called
    int last_prec = 0;
    std::vector<int32_t> user_perm;

    // device memory
    std::vector<void*> plan_allocs;  // freed at re-analyse
    DevPlan D{};
    Task* tasks_dev = nullptr;
    int32_t* lvl_sn_dev = nullptr;
    Task* stasks_dev = nullptr;               // tasks of the big-supernode solve launches
    Task* inv_tasks_dev = nullptr;            // diagonal blocks whose inverse the solves use
    std::vector<int32_t> maxf_lvl, maxp_lvl;  // per level: largest front order and pivot count
                                              // of the one-workgroup solves
    std::vector<int32_t> maxp_wave;           // per level: largest pivot count of the one-wavefront solves
    int64_t knnz = 0;
    int64_t max_sys_piv = 0;  // largest pivot count of one system
    bool fp32_fronts = false; // some trailing update belongs to a front of order >= f_mix
    int64_t device_bytes = 0;

    // solve work space
    std::vector<void*> solve_allocs;
    DevSolve S{};
    int32_t solve_cap = 0;
    // Krylov refinement work space (mixed precision), allocated on first use
    double* gm_V = nullptr;    // (GM_M + 1) blocks of N x nrhs: the Arnoldi basis
    double* gm_Z = nullptr;    // GM_M blocks of N x nrhs: the preconditioned basis M v_j
    double* gm_W = nullptr;    // N x nrhs
    DevGmres gm{};             // the small dense state, per rhs (device)
    int32_t* gm_act_host = nullptr;  // pinned copy of gm.act (eager solves)
    int32_t gm_cap = 0;
    int32_t* act_host = nullptr;  // pinned copy of the refinement flags (eager solves)
    double* shift_host = nullptr;  // pinned staging of per-system rho, delta (batch factorise)
    int32_t shift_cap = 0;
    double* shift_dev = nullptr;
    double* stats_part = nullptr;  // per-block partials of the factorisation statistics
    bool batch_shifts = false;     // the last factorisation used per-system shifts
    std::vector<int64_t> batch_col_off, batch_row_off;  // system offsets of a batch
    int32_t last_nrhs = 0;
    bool solved = false;
    // refinement state of the last solve (the handle's work space or qdmf_solve_noalloc's)
    const double* stat_berr = nullptr;
    const int32_t* stat_steps = nullptr;
    bool nopoll = false;  // qdmf_solve_noalloc: enqueue as for a graph (no host reads)

    // graph: the captured sequence in segments.  Without cuts (option graph_poll = 0) it is
    // one segment; with them, a segment starts at each decision point the eager code reads
    // on the host and runs only when its flags say that some unit still needs it.
    struct GraphSeg {
        hipGraph_t g = nullptr;
        hipGraphExec_t x = nullptr;  // null: nothing was captured in it
        const int32_t* flag = nullptr;  // run when some of flag[0 .. nflag) is nonzero (null: always)
        int32_t nflag = 0;
        size_t skip_to = 0;  // next segment when the flags are all zero
    };
    std::vector<GraphSeg> segs;
    bool capturing = false;
    bool cut_capture = false;  // capturing with cuts at the decision points
    bool capture_failed = false;
    const int32_t* cur_flag = nullptr;  // condition of the segment being captured
    int32_t cur_nflag = 0;
    std::vector<std::pair<int64_t, int64_t>> skip_pending;  // (segment, its skip target)
    int32_t* poll_host = nullptr;  // pinned flags read between segments
    int32_t poll_cap = 0;
    // what a launch of the captured graph leaves behind (set by qdmf_graph_launch)
    int32_t graph_prec = 0, graph_nrhs = 0, graph_nsolves = 0;

    // measurement: event pairs around launches of one kernel kind
    int32_t prof_kind = -1;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    double prof_flops = 0, prof_bytes = 0;

    // host copies for qdmf_symbolic
    std::vector<int32_t> h_front;
};

namespace {

void free_list(std::vector<void*>& v) {
    for (void* p : v)
        if (p) (void)hipFree(p);
    v.clear();
}

template <class T>
int dalloc(qdmf_ctx* h, std::vector<void*>& owner, T** out, int64_t count) {
    *out = nullptr;
    if (count <= 0) return 0;
    void* p = nullptr;
    if (hipMalloc(&p, sizeof(T) * (size_t)count) != hipSuccess) {
        (void)hipGetLastError();
        h->msg = "hipMalloc failed";
        return QDMF_ERR_OOM;
    }
    owner.push_back(p);
    h->device_bytes += (int64_t)(sizeof(T) * (size_t)count);
    *out = (T*)p;
    return 0;
}

template <class T>
int dupload(qdmf_ctx* h, const std::vector<T>& v, const T** out) {
    T* p = nullptr;
    int rc = dalloc(h, h->plan_allocs, &p, (int64_t)v.size());
    if (rc) return rc;
    if (!v.empty() && hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice) != hipSuccess) {
        h->msg = "hipMemcpy failed";
        return QDMF_ERR_HIP;
    }
    *out = p;
    return 0;
}

// Measurement hook: bracket one launch with an event pair when its kind is being timed.
struct ProfScope {
    qdmf_ctx* h;
    bool on;
    hipEvent_t e1 = nullptr;
    hipStream_t st;
    ProfScope(qdmf_ctx* h_, int32_t kind, double flops, double bytes, hipStream_t s = nullptr)
        : h(h_), on(false), st(s ? s : h_->stream) {
        if (h->capturing || h->prof_kind != kind) return;
        if (h->ev_used + 2 > h->ev_pool.size()) {
            for (int q = 0; q < 256; ++q) {
                hipEvent_t e;
                if (hipEventCreate(&e) != hipSuccess) return;
                h->ev_pool.push_back(e);
            }
        }
        hipEvent_t e0 = h->ev_pool[h->ev_used];
        e1 = h->ev_pool[h->ev_used + 1];
        h->ev_used += 2;
        (void)hipEventRecord(e0, st);
        h->prof_flops += flops;
        h->prof_bytes += bytes;
        on = true;
    }
    ~ProfScope() {
        if (on) (void)hipEventRecord(e1, st);
    }
};

void destroy_graph(qdmf_ctx* h) {
    for (auto& g : h->segs) {
        if (g.x) (void)hipGraphExecDestroy(g.x);
        if (g.g) (void)hipGraphDestroy(g.g);
    }
    h->segs.clear();
}

// Graph capture in segments.  seg_close ends the capture of the current segment and keeps
// it; seg_open starts the next one, run only when some of flag[0 .. n) is nonzero (flag null:
// always), and returns its index (or -1 when the capture is not cut).
void seg_close(qdmf_ctx* h) {
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(h->stream, &g) != hipSuccess || !g) {
        (void)hipGetLastError();
        h->capture_failed = true;
        if (g) (void)hipGraphDestroy(g);
        g = nullptr;
    }
    qdmf_ctx::GraphSeg sg;
    sg.g = g;
    sg.flag = h->cur_flag;
    sg.nflag = h->cur_nflag;
    size_t nn = 0;
    if (g && hipGraphGetNodes(g, nullptr, &nn) != hipSuccess) h->capture_failed = true;
    if (g && nn > 0 && hipGraphInstantiate(&sg.x, g, nullptr, nullptr, 0) != hipSuccess) {
        (void)hipGetLastError();
        sg.x = nullptr;
        h->capture_failed = true;
    }
    h->segs.push_back(sg);
}

int64_t seg_open(qdmf_ctx* h, const int32_t* flag, int32_t n) {
    if (!h->capturing || !h->cut_capture) return -1;
    seg_close(h);
    h->cur_flag = flag;
    h->cur_nflag = n;
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        h->capture_failed = true;
    }
    return (int64_t)h->segs.size();
}

// Segments q in heads that find their flags all zero continue at segment `to`.
void seg_skip(qdmf_ctx* h, const std::vector<int64_t>& heads, int64_t to) {
    for (int64_t q : heads)
        if (q >= 0) h->skip_pending.push_back({q, to});
}

int set_device(qdmf_ctx* h) {
    if (h->host_only) return QDMF_ERR_INVALID_ARG;
    return hipSetDevice(h->device) == hipSuccess ? 0 : QDMF_ERR_HIP;
}

int64_t plan_device_bytes(const Plan& P) {
    int64_t b = 0;
    b += P.front_total * 8;
    b += P.inv_total * 8 + (int64_t)P.inv_tasks.size() * sizeof(Task);
    b += (int64_t)P.tasks.size() * sizeof(Task);
    b += (int64_t)P.rows.size() * 4 + (int64_t)P.rel.size() * 4;
    b += P.kcol_ptr.empty() ? 0 : P.kcol_ptr.back() * (8 + 4 + 8);
    b += (int64_t)P.kpair.size() * 4;
    b += (int64_t)P.N * (8 * 4 + 4 + 4);
    b += (int64_t)P.acp.size() * 8 + (int64_t)P.ari.size() * 16;
    b += (int64_t)P.qfcp.size() * 8 + (int64_t)P.qfri.size() * 12 + (int64_t)P.qdiag.size() * 16 +
         (int64_t)P.qri.size() * 8;
    return b;
}

int upload_plan(qdmf_ctx* h) {
    Plan& P = h->P;
    DevPlan& D = h->D;
    D = DevPlan{};
    D.N = P.N;
    D.n = P.n;
    D.m = P.m;
    D.mode = P.mode;
    D.ns = P.ns;
    D.ub_total = P.ub_total;
    int rc = 0;
#define UP(field, vec)                          \
    if ((rc = dupload(h, P.vec, &D.field))) return rc;
    UP(sn_ptr, sn_ptr)
    UP(sn_parent, sn_parent)
    UP(sn_f, sn_f)
    UP(sn_p, sn_p)
    UP(sn_ld, sn_ld)
    UP(sn_off, sn_off)
    UP(sn_rowptr, sn_rowptr)
    UP(rows, rows)
    UP(ch_ptr, ch_ptr)
    UP(ch, ch)
    UP(rel_ptr, rel_ptr)
    UP(rel, rel)
    UP(ub_off, ub_off)
    UP(fg_ptr, fg_ptr)
    UP(fg_src, fg_src)
    UP(yoff, yoff)
    UP(inv_off, inv_off)
    UP(kcol_ptr, kcol_ptr)
    UP(kloc, kloc)
    UP(kcl, kcl)
    UP(asm_child, asm_child)
    UP(asm_col, asm_col)
    UP(ksrc, ksrc)
    UP(kpair_ptr, kpair_ptr)
    UP(kpair, kpair)
    UP(krs_ptr, krs_ptr)
    UP(krs_ent, krs_ent)
    UP(krs_other, krs_other)
    UP(primal_new, primal_new)
    UP(perm, perm)
    UP(acp, acp)
    UP(ari, ari)
    UP(arp, arp)
    UP(are, are)
    UP(acol, acol)
    UP(qfcp, qfcp)
    UP(qfri, qfri)
    UP(qfsrc, qfsrc)
    UP(qdiag, qdiag)
    UP(sys_col, sys_col)
    UP(sys_old, sys_old)
    UP(sys_new, sys_new)
    UP(sys_rng, sys_rng)
    UP(sys_piv_ptr, sys_piv_ptr)
    UP(sys_piv, sys_piv)
    UP(long_col, long_col)
    UP(long_of, long_of)
#undef UP
    {
        std::vector<int32_t> sn_sys(P.ns, 0);
        for (int32_t q = 0; q < P.ns; ++q) sn_sys[q] = P.sys_new.empty() ? 0 : P.sys_new[P.sn_ptr[q]];
        if ((rc = dupload(h, sn_sys, &D.sn_sys))) return rc;
        h->max_sys_piv = 0;
        for (int32_t q = 0; q < P.nsys; ++q)
            h->max_sys_piv = std::max<int64_t>(h->max_sys_piv, P.sys_piv_ptr[q + 1] - P.sys_piv_ptr[q]);
        h->fp32_fronts = false;
        for (const Launch& L : P.launches)
            if (L.kind == L_SYRK || L.kind == L_SYRK128)
                for (int64_t t = L.task0; t < L.task0 + L.ntask; ++t)
                    h->fp32_fronts = h->fp32_fronts || P.sn_f[P.tasks[t].s] >= h->opt.f_mix;
    }
    D.nlong = (int32_t)P.long_col.size();
    D.nsys = P.nsys;
    D.has_q = P.has_q ? 1 : 0;
    const Task* tk = nullptr;
    if ((rc = dupload(h, P.tasks, &tk))) return rc;
    h->tasks_dev = const_cast<Task*>(tk);
    const int32_t* ls = nullptr;
    if ((rc = dupload(h, P.lvl_sn, &ls))) return rc;
    h->lvl_sn_dev = const_cast<int32_t*>(ls);
    const Task* stk = nullptr;
    if ((rc = dupload(h, P.stasks, &stk))) return rc;
    h->stasks_dev = const_cast<Task*>(stk);
    const Task* itk = nullptr;
    if ((rc = dupload(h, P.inv_tasks, &itk))) return rc;
    h->inv_tasks_dev = const_cast<Task*>(itk);
    h->knnz = P.kcol_ptr.empty() ? 0 : P.kcol_ptr.back();
    const int64_t N = P.N;
    if ((rc = dalloc(h, h->plan_allocs, &D.front, P.front_total))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.kval, h->knnz))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.linv, P.inv_total))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.aval, (int64_t)P.ari.size()))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.colabs, P.n))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.rowabs, P.m))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.qval, (int64_t)P.qri.size()))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.qoff, P.has_q ? P.n : 0))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.dinv, P.n))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.rowsum, N))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.dval, N))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.doff, N))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.ptype, N))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.edyn, N))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.pflag, N))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.zskip, N))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.lperm, N))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.lpinv, N))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.sc, 1))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.st, 1))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.knorm_sys, P.nsys))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.rho_sys, P.nsys))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.delta_sys, P.nsys))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.inertia_sys, (int64_t)3 * P.nsys))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &D.redo, (int64_t)P.nsys + 1))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &h->shift_dev, (int64_t)2 * P.nsys))) return rc;
    if ((rc = dalloc(h, h->plan_allocs, &h->stats_part, (int64_t)10 * factor_stats_blocks(P.N)))) return rc;
    // largest front (dynamic LDS of the one-workgroup solve kernels) and pivot count (kernel
    // variant) per level, over the supernodes those kernels solve
    h->maxf_lvl.assign(P.nlevels, 1);
    h->maxp_lvl.assign(P.nlevels, 1);
    h->maxp_wave.assign(P.nlevels, 1);
    for (int32_t l = 0; l < P.nlevels; ++l) {
        for (int64_t q = P.lvl_ptr[l]; q < P.lvl_ptr[l] + P.lvl_wave[l]; ++q)
            h->maxp_wave[l] = std::max(h->maxp_wave[l], P.sn_p[P.lvl_sn[q]]);
        for (int64_t q = P.lvl_ptr[l] + P.lvl_wave[l]; q < P.lvl_ptr[l] + P.lvl_small[l]; ++q) {
            h->maxf_lvl[l] = std::max(h->maxf_lvl[l], P.sn_f[P.lvl_sn[q]]);
            h->maxp_lvl[l] = std::max(h->maxp_lvl[l], P.sn_p[P.lvl_sn[q]]);
        }
    }
    if (hipDeviceSynchronize() != hipSuccess) return QDMF_ERR_HIP;
    return 0;
}

// Device work space of the solves.  One layout serves the allocated work space of qdmf_solve
// and the fixed array of qdmf_solve_noalloc: a first pass with base == nullptr sizes it, a
// second assigns the arrays (each on a 256-byte boundary).
struct Carve {
    char* base = nullptr;
    int64_t off = 0;
    template <class T>
    T* take(int64_t n) {
        off = (off + 255) & ~(int64_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += (int64_t)sizeof(T) * std::max<int64_t>(n, 1);
        return p;
    }
};

void layout_solve(const qdmf_ctx* h, int32_t nrhs, Carve& c, DevSolve& S) {
    const int64_t N = h->P.N;
    S.nrhs = nrhs;
    S.nblk = (int32_t)((N + 255) / 256);
    S.b = c.take<double>(N * nrhs);
    S.x = c.take<double>(N * nrhs);
    S.xbak = c.take<double>(N * nrhs);
    S.r = c.take<double>(N * nrhs);
    S.d = c.take<double>(N * nrhs);
    S.xw = c.take<double>(N * nrhs);
    S.ub = c.take<double>(std::max<int64_t>(1, h->P.ub_total) * nrhs);
    S.part = c.take<double>((int64_t)4 * S.nblk * nrhs);
    const int64_t units = (int64_t)nrhs * h->P.nsys;
    S.berr = c.take<double>(4 * units);
    S.active = c.take<int32_t>(units);
    S.steps = c.take<int32_t>(units);
    S.ract = c.take<int32_t>(nrhs);
    S.ytot = h->P.ytotal;
    S.Y = c.take<double>(std::max<int64_t>(1, h->P.ytotal) * nrhs);
    S.P = c.take<double>(std::max<int64_t>(1, h->P.ppart_max) * SOLVE_BLOCK * nrhs);
    S.lsum = c.take<double>(std::max<int64_t>(1, (int64_t)h->P.long_col.size()) * 2 * nrhs);
}

// Krylov work space for cap right-hand sides (mixed-precision refinement).
void layout_gmres(const qdmf_ctx* h, int32_t cap, Carve& c, double*& V, double*& Z, double*& W, DevGmres& G) {
    const int64_t N = h->P.N;
    const int64_t nu = (int64_t)cap * h->P.nsys;  // refinement units
    V = c.take<double>((int64_t)(GM_M + 1) * N * cap);
    Z = c.take<double>((int64_t)GM_M * N * cap);
    W = c.take<double>(N * cap);
    G.h1 = c.take<double>((GM_M + 1) * nu);
    G.h2 = c.take<double>((GM_M + 1) * nu);
    G.nrm = c.take<double>(nu);
    G.beta = c.take<double>(nu);
    G.g = c.take<double>((GM_M + 1) * nu);
    G.cs = c.take<double>(GM_M * nu);
    G.sn = c.take<double>(GM_M * nu);
    G.R = c.take<double>((int64_t)GM_M * GM_M * nu);
    G.y = c.take<double>(GM_M * nu);
    G.kr = c.take<int32_t>(nu);
    G.act = c.take<int32_t>(nu);
    G.ract = c.take<int32_t>(cap);
}

int ensure_solve(qdmf_ctx* h, int32_t nrhs) {
    if (nrhs <= h->solve_cap) {
        h->S.nrhs = nrhs;
        return 0;
    }
    free_list(h->solve_allocs);
    destroy_graph(h);
    h->gm_V = h->gm_Z = h->gm_W = nullptr;
    h->gm = DevGmres{};
    h->gm_cap = 0;
    DevSolve& S = h->S;
    Carve c;
    layout_solve(h, nrhs, c, S);
    int rc = 0;
    if ((rc = dalloc(h, h->solve_allocs, &c.base, c.off))) return rc;
    c.off = 0;
    layout_solve(h, nrhs, c, S);
    const int64_t units = (int64_t)nrhs * h->P.nsys;
    if (h->act_host) (void)hipHostFree(h->act_host);
    h->act_host = nullptr;
    if (hipHostMalloc((void**)&h->act_host, sizeof(int32_t) * units, hipHostMallocDefault) != hipSuccess) {
        h->act_host = nullptr;
        return QDMF_ERR_OOM;
    }
    h->solve_cap = nrhs;
    S.nrhs = nrhs;
    return 0;
}

PivotParams pivot_params(const qdmf_ctx* h, int32_t prec) {
    PivotParams pp;
    pp.alpha = h->opt.alpha;
    pp.eps_lift = h->opt.eps_lift;
    pp.tau_big = h->opt.tau_big;
    pp.presort = h->opt.presort;
    // a mixed factorisation without any front of order >= f_mix computes what FP64 does
    pp.mixed = prec == QDMF_MIXED && h->fp32_fronts;
    pp.f_mix = h->opt.f_mix;
    pp.mixed_check = h->opt.mixed_check;
    return pp;
}

// The plan's factorisation launches in order.  Launches marked for the second stream start
// after the last pivot window enqueued before them; a launch marked to wait, and every
// assembly, small-front or finalize step, first waits for the second stream's work so far;
// the second stream is joined back before returning, so the caller's stream (and a graph
// captured on it) holds everything.
void enqueue_launches(qdmf_ctx* h, const DevPlan& D, const PivotParams& pp, bool count_work) {
    bool pending = false;  // second-stream work not yet joined
    for (const Launch& L : h->P.launches) {
        hipStream_t st = h->stream;
        if (L.stream == 1) {
            st = h->stream2;
            (void)hipStreamWaitEvent(st, h->ev_win, 0);
        } else if (pending && (L.wait || L.kind == L_SMALL || L.kind == L_ASSEMBLE || L.kind == L_FINALIZE ||
                               L.nfin > 0)) {
            (void)hipStreamWaitEvent(h->stream, h->ev_s2, 0);
            pending = false;
        }
        {
            ProfScope ps(h, L.kind, count_work ? L.flops : 0.0, count_work ? L.bytes : 0.0, st);
            launch_factor_step(D, L, h->tasks_dev, pp, st);
        }
        if (L.stream == 1) {
            (void)hipEventRecord(h->ev_s2, st);
            pending = true;
        } else if (L.kind == L_WINDOW && h->ev_win) {
            (void)hipEventRecord(h->ev_win, h->stream);
        }
    }
    if (pending) (void)hipStreamWaitEvent(h->stream, h->ev_s2, 0);
}

// The second stream and its events, when the plan has launches for it (each object is
// created once and kept until the handle is destroyed).
int ensure_stream2(qdmf_ctx* h) {
    bool any = false;
    for (const Launch& L : h->P.launches) any = any || L.stream == 1;
    if (!any) return 0;
    if (!h->stream2 && hipStreamCreateWithFlags(&h->stream2, hipStreamNonBlocking) != hipSuccess) {
        h->stream2 = nullptr;
        return QDMF_ERR_HIP;
    }
    if (!h->ev_win && hipEventCreateWithFlags(&h->ev_win, hipEventDisableTiming) != hipSuccess) {
        h->ev_win = nullptr;
        return QDMF_ERR_HIP;
    }
    if (!h->ev_s2 && hipEventCreateWithFlags(&h->ev_s2, hipEventDisableTiming) != hipSuccess) {
        h->ev_s2 = nullptr;
        return QDMF_ERR_HIP;
    }
    return 0;
}

// rho_dev, delta_dev: per-system shifts on the device (nsys each), or NULL (rho, delta for all)
void enqueue_factorise(qdmf_ctx* h, const double* theta, double rho, double delta, const double* rho_dev,
                       const double* delta_dev, int32_t prec) {
    const PivotParams pp = pivot_params(h, prec);
    launch_theta(h->D, theta, rho, delta, rho_dev, delta_dev, h->stream);
    launch_values_n(h->D, h->knnz, h->stream);
    launch_knorm(h->D, h->stream);
    enqueue_launches(h, h->D, pp, true);
    launch_inv(h->D, h->inv_tasks_dev, (int64_t)h->P.inv_tasks.size(), h->stream);
    launch_factor_stats(h->D, pp, h->stats_part, h->stream);
    if (!pp.mixed || pp.mixed_check == 0) return;
    // Mixed precision: the systems whose FP32 updates broke down are factorised again in FP64
    // (the same launches, gated to those systems' supernodes).  Eager execution reads the count
    // and skips the second pass when it is zero; a captured graph always holds it.
    launch_mixed_check(h->D, pp, h->max_sys_piv, h->stream);
    const int64_t redo_seg = seg_open(h, h->D.redo + h->P.nsys, 1);
    if (!h->capturing) {
        int32_t nredo = 0;
        if (hipMemcpyAsync(&nredo, h->D.redo + h->P.nsys, sizeof(nredo), hipMemcpyDeviceToHost, h->stream) !=
                hipSuccess ||
            hipStreamSynchronize(h->stream) != hipSuccess)
            nredo = 1;  // unknown: take the safe path
        if (nredo == 0) return;
    }
    DevPlan G = h->D;
    G.gate = h->D.redo;
    const PivotParams p64 = pivot_params(h, QDMF_FP64);
    enqueue_launches(h, G, p64, false);
    launch_inv(G, h->inv_tasks_dev, (int64_t)h->P.inv_tasks.size(), h->stream);
    launch_factor_stats(h->D, p64, h->stats_part, h->stream);
    if (redo_seg >= 0) seg_skip(h, {redo_seg}, seg_open(h, nullptr, 0));
}

// (L D L^T)^{-1} src -> dst, level by level (forward leaves first, backward roots first).
// active: NULL, or per refinement unit (rhs x system; a batch gates the kernels by "some system
// of the rhs still refines") when per_rhs is false, or already per rhs when it is true.
void enqueue_ldlt_solve(qdmf_ctx* h, const double* src, double* dst, const int32_t* active, bool per_rhs = false) {
    const Plan& P = h->P;
    const DevSolve& S = h->S;
    hipStream_t st = h->stream;
    if (P.nsys > 1 && active && !per_rhs) active = S.ract;
    launch_permute(h->D, S, src, active, st);
    // per level: the supernodes of fronts up to 64 rows one per wavefront, the other small ones
    // one per workgroup, then the steps of the big ones
    auto level = [&](bool fwd, int32_t l) {
        const int64_t b = P.lvl_ptr[l];
        const int32_t nw = P.lvl_wave[l];
        launch_solve_level(fwd, h->D, S, h->lvl_sn_dev, b, (unsigned)nw, 64, h->maxp_wave[l], active, st);
        launch_solve_level(fwd, h->D, S, h->lvl_sn_dev, b + nw, (unsigned)(P.lvl_small[l] - nw), h->maxf_lvl[l],
                           h->maxp_lvl[l], active, st);
    };
    for (int32_t l = 0; l < P.nlevels; ++l) {
        ProfScope ps(h, QDMF_K_FWD, P.lvl_solve_flops[l] * S.nrhs, P.lvl_solve_bytes[l] * S.nrhs);
        level(true, l);
        for (int64_t q = P.fwd_ptr[l]; q < P.fwd_ptr[l + 1]; ++q)
            launch_big_solve(h->D, S, P.fwd_plan[q], h->stasks_dev, active, st);
    }
    for (int32_t l = P.nlevels - 1; l >= 0; --l) {
        ProfScope ps(h, QDMF_K_BWD, P.lvl_solve_flops[l] * S.nrhs, P.lvl_solve_bytes[l] * S.nrhs);
        level(false, l);
        for (int64_t q = P.bwd_ptr[l]; q < P.bwd_ptr[l + 1]; ++q)
            launch_big_solve(h->D, S, P.bwd_plan[q], h->stasks_dev, active, st);
    }
    launch_unpermute(h->D, S, dst, active, st);
}

// ---- FP64 refinement with a Krylov correction (mixed precision)
// Each correction d of K_static d = r comes from GMRES on K_static M, right-preconditioned by
// the mixed-precision factor M = (L D L^T)^{-1}, with the preconditioned vectors z_j = M v_j
// kept (so d = Z y needs no further solve): it minimises the FP64 residual ||r - K d||_2 over the
// Krylov space, and still converges when the FP32 updates leave ||I - K M|| above one, where
// plain refinement d = M r diverges.  GM_M steps at most per correction (restarted by the
// refinement loop), classical Gram-Schmidt applied twice; the Hessenberg reduction, the stop
// flags and the small triangular solve run on the device.  Every step is enqueued when the
// sequence is captured into a graph (its kernels return at once for converged right-hand
// sides); eager solves read the device's flags before each further step and stop launching
// once none is left, which skips only launches that would have done nothing (the results are
// the same bit for bit).
constexpr double GM_TOL = 1e-6;  // reduction of ||r - K d||_2 that ends a correction

int ensure_gmres(qdmf_ctx* h) {
    const int32_t nr = h->S.nrhs;
    if (h->gm_V && h->gm_cap >= nr) return 0;
    const int32_t cap = std::max(nr, h->solve_cap);
    Carve c;
    layout_gmres(h, cap, c, h->gm_V, h->gm_Z, h->gm_W, h->gm);
    int rc = 0;
    if ((rc = dalloc(h, h->solve_allocs, &c.base, c.off))) return rc;
    c.off = 0;
    layout_gmres(h, cap, c, h->gm_V, h->gm_Z, h->gm_W, h->gm);
    if (h->gm_act_host) (void)hipHostFree(h->gm_act_host);
    h->gm_act_host = nullptr;
    if (hipHostMalloc((void**)&h->gm_act_host, sizeof(int32_t) * cap, hipHostMallocDefault) != hipSuccess) {
        h->gm_act_host = nullptr;
        return QDMF_ERR_OOM;
    }
    h->gm_cap = cap;
    return 0;
}

// S.d = the Krylov correction of K_static d = S.r for every refinement unit that continues.
// The work space must exist (ensure_gmres) before a capture starts: nothing is allocated here.
int enqueue_gmres_correction(qdmf_ctx* h) {
    DevSolve& S = h->S;
    const int32_t nr = S.nrhs, ns = h->P.nsys, nu = nr * ns;
    const int64_t N = h->P.N;
    hipStream_t st = h->stream;
    if (!h->gm_V || h->gm_cap < nr) return QDMF_ERR_INVALID_ARG;
    const DevGmres& G = h->gm;
    const DevPlan& D = h->D;
    auto Vb = [&](int j) { return h->gm_V + (int64_t)j * N * nr; };
    auto Zb = [&](int j) { return h->gm_Z + (int64_t)j * N * nr; };
    launch_dots(D, S.r, 1, S.r, G.nrm, nr, nullptr, st);
    launch_gm_start(G, S.active, nu, st);  // per unit: the refinement continues and r != 0
    launch_gm_gate(G, nr, ns, st);  // per rhs: some unit takes the first step
    launch_vscale(D, S.r, G.nrm, Vb(0), nr, G.act, st);
    std::vector<int64_t> steps;  // cut capture: the segments of Krylov steps 1 ..
    for (int j = 0; j < GM_M; ++j) {
        if (j > 0) steps.push_back(seg_open(h, G.ract, nr));
        if (!h->capturing && !h->nopoll && j > 0) {
            if (hipMemcpyAsync(h->gm_act_host, G.ract, sizeof(int32_t) * nr, hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                return QDMF_ERR_HIP;
            bool any = false;
            for (int r = 0; r < nr; ++r) any = any || h->gm_act_host[r] != 0;
            if (!any) break;
        }
        enqueue_ldlt_solve(h, Vb(j), Zb(j), G.ract, true);  // z_j = M v_j
        launch_matvec(D, Zb(j), h->gm_W, nr, S.lsum, G.ract, st);  // w = K z_j
        launch_dots(D, h->gm_V, j + 1, h->gm_W, G.h1, nr, G.act, st);
        launch_vcombine(D, h->gm_V, j + 1, G.h1, h->gm_W, nr, true, G.act, nullptr, st);
        launch_dots(D, h->gm_V, j + 1, h->gm_W, G.h2, nr, G.act, st);
        launch_vcombine(D, h->gm_V, j + 1, G.h2, h->gm_W, nr, true, G.act, nullptr, st);
        launch_dots(D, h->gm_W, 1, h->gm_W, G.nrm, nr, G.act, st);
        launch_vscale(D, h->gm_W, G.nrm, Vb(j + 1), nr, G.act, st);
        launch_gm_rotate(G, j, nr, ns, GM_TOL, st);
    }
    if (h->capturing && h->cut_capture) seg_skip(h, steps, seg_open(h, nullptr, 0));
    launch_gm_solve(G, nu, st);
    launch_vcombine(D, h->gm_Z, GM_M, G.y, S.d, nr, false, nullptr, G.kr, st);  // d = Z y per unit
    return 0;
}

// The refinement of a mixed factorisation takes Krylov corrections when its factor holds FP32
// products; without any front of order >= f_mix the factor is FP64's, and so is the correction.
bool krylov_refine(const qdmf_ctx* h) {
    return h->last_prec == QDMF_MIXED && h->fp32_fronts && h->opt.max_refine_mixed > 0;
}

void enqueue_solve(qdmf_ctx* h, const double* r7, const double* r1, double* dx, double* dy) {
    const DevPlan& D = h->D;
    const DevSolve& S = h->S;
    const bool mixed = h->last_prec == QDMF_MIXED;
    const bool krylov = krylov_refine(h);
    const double target = mixed ? h->opt.target_berr_mixed : h->opt.target_berr;
    const int max_steps = mixed ? h->opt.max_refine_mixed : h->opt.max_refine;
    hipStream_t st = h->stream;
    if (krylov && !h->capturing && !h->nopoll && ensure_gmres(h)) return;  // no work space: no refinement
    launch_rhs(D, S, r7, r1, st);
    enqueue_ldlt_solve(h, S.b, S.x, nullptr);
    launch_residual(D, S, S.x, st);
    launch_berr_steps(D, S, 0, target, max_steps, st);
    std::vector<int64_t> passes;  // cut capture: the segments of the refinement passes
    for (int it = 0; it < max_steps; ++it) {
        passes.push_back(seg_open(h, S.active, (int32_t)((int64_t)S.nrhs * h->P.nsys)));
        // Eager solves look at the refinement flags and stop launching once every
        // right-hand side has met the target; a captured graph (and qdmf_solve_noalloc)
        // keeps all passes and the kernels of a finished right-hand side return at once.
        if (!h->capturing && !h->nopoll) {
            const int64_t units = (int64_t)S.nrhs * h->P.nsys;
            if (hipMemcpyAsync(h->act_host, S.active, sizeof(int32_t) * units, hipMemcpyDeviceToHost, st) !=
                    hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess)
                break;
            bool any = false;
            for (int64_t u = 0; u < units; ++u) any = any || h->act_host[u] != 0;
            if (!any) break;
        }
        launch_refine_begin(D, S, st);
        if (krylov) {
            if (enqueue_gmres_correction(h)) break;
        } else {
            enqueue_ldlt_solve(h, S.r, S.d, S.active);
        }
        launch_refine_update(D, S, st);
        launch_residual(D, S, S.x, st);
        launch_berr_steps(D, S, 1, target, max_steps, st);
    }
    if (h->capturing && h->cut_capture) seg_skip(h, passes, seg_open(h, nullptr, 0));
    launch_recover(D, S, r7, dx, dy, st);
    h->stat_berr = S.berr;
    h->stat_steps = S.steps;
}

// Work space of qdmf_solve_noalloc: a fixed array in device memory, one copy per GPU, held
// until the process ends.  Host code never passes its name to a kernel or a copy: it uses the
// address that hipGetSymbolAddress returns with the GPU current (scratch_addr).
constexpr int NOALLOC_MAX_DEVICES = 64;
static __device__ __align__(256) unsigned char scratch[QDMF_NOALLOC_SCRATCH_BYTES];
std::mutex scratch_mu;
void* scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// Looks up (once per device, that device current) the device address of this GPU's copy.
int scratch_lookup(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return QDMF_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_ptr[device]) return 0;
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return QDMF_ERR_HIP;
    }
    scratch_ptr[device] = p;
    return 0;
}

void* scratch_addr(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    return scratch_ptr[device];
}

}  // namespace

extern "C" {

void qdmf_default_options(qdmf_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->nb = 64;
    o->alpha = (1.0 + std::sqrt(17.0)) / 8.0;
    o->eps_lift = 2.220446049250313e-16;
    o->presort = 1;
    o->max_refine = 2;
    o->max_refine_mixed = 3;
    o->target_berr = 1e-12;
    o->target_berr_mixed = 1e-10;
    o->tau_big = 1e-8;
    o->ordering = QDMF_ORDER_AUTO;
    o->amalgamate = 1;
    o->f_mix = 1024;
    o->small_front = 64;
    o->mem_cap_bytes = 0;
    o->split_solve_front = 1024;
    o->syrk_group_front = 1024;
    o->syrk_group = 4;
    o->syrk_tile_front = 0;
    o->mixed_check = 2;
    o->lookahead_front = 0;
    o->graph_poll = 1;
}

int qdmf_create(qdmf_handle* out, int device, void* hip_stream, const qdmf_options* opt) {
    if (!out) return QDMF_ERR_INVALID_ARG;
    *out = nullptr;
    qdmf_ctx* h = new qdmf_ctx();
    if (opt) h->opt = *opt;
    else qdmf_default_options(&h->opt);
    if (h->opt.nb != 64 || h->opt.small_front < 1 || h->opt.small_front > 64 || h->opt.split_solve_front < 1 ||
        h->opt.syrk_group_front < 0 || h->opt.syrk_group < 1 || h->opt.syrk_group > SYRK_GROUP_MAX ||
        h->opt.syrk_tile_front < 0 || h->opt.mixed_check < 0 || h->opt.mixed_check > 3 ||
        h->opt.lookahead_front < 0 ||
        h->opt.max_refine < 0 ||
        h->opt.max_refine_mixed < 0 || h->opt.ordering < QDMF_ORDER_AMD || h->opt.ordering > QDMF_ORDER_AUTO) {
        delete h;
        return QDMF_ERR_INVALID_ARG;
    }
    h->device = device;
    h->host_only = device < 0;
    h->stream = (hipStream_t)hip_stream;
    if (!h->host_only) {
        int count = 0;
        if (hipGetDeviceCount(&count) != hipSuccess || device >= count || hipSetDevice(device) != hipSuccess) {
            (void)hipGetLastError();
            delete h;
            return QDMF_ERR_HIP;
        }
        // the allocation-free solve's work space on this GPU (a failure only disables that call)
        (void)scratch_lookup(device);
    }
    *out = h;
    return 0;
}

int qdmf_set_stream(qdmf_handle h, void* s) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (h->stream != (hipStream_t)s) destroy_graph(h);
    h->stream = (hipStream_t)s;
    return 0;
}

namespace {

int analyse_impl(qdmf_handle h, int32_t m, int32_t n, const int64_t* colptr, const int32_t* rowidx, int32_t mode,
                 const int32_t* user_perm, int32_t nsys, const int64_t* col_off, const int64_t* row_off,
                 const int64_t* q_colptr = nullptr, const int32_t* q_rowidx = nullptr) {
    if (!h->host_only) {
        int rc = set_device(h);
        if (rc) return rc;
        (void)hipStreamSynchronize(h->stream);
    }
    destroy_graph(h);
    free_list(h->solve_allocs);
    free_list(h->plan_allocs);
    h->solve_cap = 0;
    h->analysed = h->have_matrix = h->factorised = h->solved = false;
    h->have_hessian = false;
    h->device_bytes = 0;
    AnalyseOptions ao;
    ao.ordering = h->opt.ordering;
    for (int a = 0; a < 3; ++a) ao.grid[a] = h->opt.grid[a];
    ao.amalgamate = h->opt.amalgamate;
    ao.small_front = h->opt.small_front;
    ao.split_solve_front = h->opt.split_solve_front;
    ao.syrk_group_front = h->opt.syrk_group_front;
    ao.syrk_group = h->opt.syrk_group;
    ao.syrk_tile_front = h->opt.syrk_tile_front;
    ao.lookahead_front = h->opt.lookahead_front;
    ao.f_mix = h->opt.f_mix;
    ao.user_perm = user_perm;
    ao.nsys = nsys;
    ao.col_off = col_off;
    ao.row_off = row_off;
    ao.q_colptr = q_colptr;
    ao.q_rowidx = q_rowidx;
    if (h->opt.ordering == QDMF_ORDER_USER && !user_perm) return QDMF_ERR_INVALID_ARG;
    int rc = build_plan(m, n, colptr, rowidx, mode, ao, h->P, h->msg);
    if (rc) return rc;
    const int64_t need = plan_device_bytes(h->P);
    if (h->opt.mem_cap_bytes > 0 && need > h->opt.mem_cap_bytes) {
        h->msg = "memory plan exceeds the cap";
        return QDMF_ERR_OOM;
    }
    h->h_front = h->P.sn_f;
    if (!h->host_only) {
        rc = upload_plan(h);
        if (!rc) rc = ensure_stream2(h);
        if (rc) {
            free_list(h->plan_allocs);
            return rc;
        }
    }
    h->analysed = true;
    return 0;
}

}  // namespace

int qdmf_analyse(qdmf_handle h, int32_t m, int32_t n, const int64_t* colptr, const int32_t* rowidx,
                 int32_t mode, const int32_t* user_perm) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    h->batch_col_off.clear();
    h->batch_row_off.clear();
    return analyse_impl(h, m, n, colptr, rowidx, mode, user_perm, 1, nullptr, nullptr);
}

int qdmf_analyse_qp(qdmf_handle h, int32_t m, int32_t n, const int64_t* colptr, const int32_t* rowidx,
                    const int64_t* q_colptr, const int32_t* q_rowidx, const int32_t* user_perm) {
    if (!h || !q_colptr) return QDMF_ERR_INVALID_ARG;
    h->batch_col_off.clear();
    h->batch_row_off.clear();
    return analyse_impl(h, m, n, colptr, rowidx, QDMF_AS, user_perm, 1, nullptr, nullptr, q_colptr, q_rowidx);
}

int qdmf_batch_analyse(qdmf_handle h, int32_t count, const int32_t* m, const int32_t* n,
                       const int64_t* const* colptr, const int32_t* const* rowidx, int32_t mode) {
    if (!h || count < 1 || !m || !n || !colptr || !rowidx) return QDMF_ERR_INVALID_ARG;
    if (h->opt.ordering == QDMF_ORDER_USER || h->opt.ordering == QDMF_ORDER_GRID_ND) return QDMF_ERR_INVALID_ARG;
    std::vector<int64_t> coff(count + 1, 0), roff(count + 1, 0);
    int64_t nnz = 0;
    for (int32_t q = 0; q < count; ++q) {
        if (m[q] < 0 || n[q] < 0 || !colptr[q] || (n[q] > 0 && !rowidx[q] && colptr[q][n[q]] > 0))
            return QDMF_ERR_INVALID_ARG;
        coff[q + 1] = coff[q] + n[q];
        roff[q + 1] = roff[q] + m[q];
        nnz += colptr[q][n[q]] - colptr[q][0];
    }
    if (coff[count] > INT32_MAX || roff[count] > INT32_MAX) return QDMF_ERR_INDEX_OVERFLOW;
    // the block-diagonal pattern: system q's column j is column coff[q] + j, its row i row roff[q] + i
    std::vector<int64_t> cp(coff[count] + 1, 0);
    std::vector<int32_t> ri;
    ri.reserve(nnz);
    for (int32_t q = 0; q < count; ++q)
        for (int32_t j = 0; j < n[q]; ++j) {
            for (int64_t e = colptr[q][j]; e < colptr[q][j + 1]; ++e) {
                const int32_t r = rowidx[q][e];
                if (r < 0 || r >= m[q]) return QDMF_ERR_INVALID_ARG;
                ri.push_back((int32_t)(roff[q] + r));
            }
            cp[coff[q] + j + 1] = (int64_t)ri.size();
        }
    h->batch_col_off = coff;
    h->batch_row_off = roff;
    const int rc = analyse_impl(h, (int32_t)roff[count], (int32_t)coff[count], cp.data(), ri.data(), mode, nullptr,
                                count, coff.data(), roff.data());
    if (rc) {
        h->batch_col_off.clear();
        h->batch_row_off.clear();
    }
    return rc;
}

int qdmf_batch_offsets(qdmf_handle h, int64_t* row_off, int64_t* col_off) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->analysed) return QDMF_ERR_NOT_ANALYSED;
    const int32_t ns = h->P.nsys;
    for (int32_t q = 0; q <= ns; ++q) {
        if (row_off) row_off[q] = h->batch_row_off.empty() ? (q ? h->P.m : 0) : h->batch_row_off[q];
        if (col_off) col_off[q] = h->batch_col_off.empty() ? (q ? h->P.n : 0) : h->batch_col_off[q];
    }
    return 0;
}

int qdmf_symbolic(qdmf_handle h, qdmf_symbolic_info* out) {
    if (!h || !out) return QDMF_ERR_INVALID_ARG;
    if (!h->analysed) return QDMF_ERR_NOT_ANALYSED;
    const Plan& P = h->P;
    out->N = P.N;
    out->nsuper = P.ns;
    out->nlevels = P.nlevels;
    out->max_front = P.max_front;
    out->nnz_l = P.nnz_l;
    out->nnz_k = P.kcol_ptr.empty() ? 0 : P.kcol_ptr.back();
    out->flops_fact = P.flops_fact;
    out->flops_solve = P.flops_solve;
    out->device_bytes = h->host_only ? plan_device_bytes(P) : h->device_bytes;
    out->front_bytes = P.front_total * 8;
    out->perm = P.perm.data();
    out->sn_ptr = P.sn_ptr.data();
    out->sn_parent = P.sn_parent.data();
    out->sn_front = P.sn_f.data();
    out->sn_level = P.sn_level.data();
    return 0;
}

int qdmf_set_matrix(qdmf_handle h, const double* a_val, int32_t on_device) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->analysed) return QDMF_ERR_NOT_ANALYSED;
    if (h->host_only) return QDMF_ERR_INVALID_ARG;
    const int64_t nnz = (int64_t)h->P.ari.size();
    if (nnz > 0 && !a_val) return QDMF_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    if (nnz > 0) {
        hipError_t e = hipMemcpyAsync(h->D.aval, a_val, sizeof(double) * (size_t)nnz,
                                      on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream);
        if (e != hipSuccess) return QDMF_ERR_HIP;
    }
    launch_matrix_norms(h->D, h->stream);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    h->have_matrix = true;
    h->factorised = false;
    return 0;
}

int qdmf_set_hessian(qdmf_handle h, const double* q_val, int32_t on_device) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->analysed) return QDMF_ERR_NOT_ANALYSED;
    if (h->host_only || !h->P.has_q) return QDMF_ERR_INVALID_ARG;
    const int64_t nnz = (int64_t)h->P.qri.size();
    if (nnz > 0 && !q_val) return QDMF_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    if (nnz > 0 && hipMemcpyAsync(h->D.qval, q_val, sizeof(double) * (size_t)nnz,
                                  on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, h->stream) != hipSuccess)
        return QDMF_ERR_HIP;
    launch_hessian_norms(h->D, h->stream);
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    h->have_hessian = true;
    h->factorised = false;
    return 0;
}

int qdmf_factorise(qdmf_handle h, const double* theta_dev, double rho, double delta, int32_t prec) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->analysed) return QDMF_ERR_NOT_ANALYSED;
    if (!h->have_matrix || (h->P.has_q && !h->have_hessian)) return QDMF_ERR_NO_MATRIX;
    if (h->host_only || (!theta_dev && h->P.n > 0) || !(rho >= 0) || !(delta >= 0) || !std::isfinite(rho) ||
        !std::isfinite(delta) || (prec != QDMF_FP64 && prec != QDMF_MIXED))
        return QDMF_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    if (h->P.N > 0) enqueue_factorise(h, theta_dev, rho, delta, nullptr, nullptr, prec);  // an empty system: nothing to do
    if (hipGetLastError() != hipSuccess) return QDMF_ERR_HIP;
    h->last_prec = prec;
    h->factorised = true;
    h->solved = false;
    return 0;
}

int qdmf_batch_factorise(qdmf_handle h, const double* theta_dev, const double* rho, const double* delta,
                         int32_t prec) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->analysed) return QDMF_ERR_NOT_ANALYSED;
    if (!h->have_matrix) return QDMF_ERR_NO_MATRIX;
    const int32_t ns = h->P.nsys;
    if (h->host_only || (!theta_dev && h->P.n > 0) || !rho || !delta || (prec != QDMF_FP64 && prec != QDMF_MIXED))
        return QDMF_ERR_INVALID_ARG;
    for (int32_t q = 0; q < ns; ++q)
        if (!(rho[q] >= 0) || !(delta[q] >= 0) || !std::isfinite(rho[q]) || !std::isfinite(delta[q]))
            return QDMF_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    // the staging buffer may still feed an earlier copy on the stream: wait for it
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    if (h->shift_cap < ns) {
        if (h->shift_host) (void)hipHostFree(h->shift_host);
        h->shift_cap = 0;
        if (hipHostMalloc((void**)&h->shift_host, sizeof(double) * 2 * ns, hipHostMallocDefault) != hipSuccess) {
            h->shift_host = nullptr;
            return QDMF_ERR_OOM;
        }
        h->shift_cap = ns;
    }
    for (int32_t q = 0; q < ns; ++q) {
        h->shift_host[q] = rho[q];
        h->shift_host[ns + q] = delta[q];
    }
    if (hipMemcpyAsync(h->shift_dev, h->shift_host, sizeof(double) * 2 * ns, hipMemcpyHostToDevice, h->stream) !=
        hipSuccess)
        return QDMF_ERR_HIP;
    if (h->P.N > 0) enqueue_factorise(h, theta_dev, rho[0], delta[0], h->shift_dev, h->shift_dev + ns, prec);
    if (hipGetLastError() != hipSuccess) return QDMF_ERR_HIP;
    h->last_prec = prec;
    h->factorised = true;
    h->solved = false;
    return 0;
}

int qdmf_batch_factorise_dev(qdmf_handle h, const double* theta_dev, const double* rho_dev,
                             const double* delta_dev, int32_t prec) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->analysed) return QDMF_ERR_NOT_ANALYSED;
    if (!h->have_matrix || (h->P.has_q && !h->have_hessian)) return QDMF_ERR_NO_MATRIX;
    if (h->host_only || (!theta_dev && h->P.n > 0) || !rho_dev || !delta_dev ||
        (prec != QDMF_FP64 && prec != QDMF_MIXED))
        return QDMF_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    if (h->P.N > 0) enqueue_factorise(h, theta_dev, 0.0, 0.0, rho_dev, delta_dev, prec);
    if (hipGetLastError() != hipSuccess) return QDMF_ERR_HIP;
    h->last_prec = prec;
    h->factorised = true;
    h->solved = false;
    return 0;
}

int qdmf_batch_stats(qdmf_handle h, int64_t* inertia, double* berr_nw, int32_t* steps) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->factorised) return QDMF_ERR_NOT_FACTORISED;
    if (set_device(h)) return QDMF_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    const size_t ns = (size_t)h->P.nsys;
    if (inertia && hipMemcpy(inertia, h->D.inertia_sys, sizeof(int64_t) * 3 * ns, hipMemcpyDeviceToHost) != hipSuccess)
        return QDMF_ERR_HIP;
    if (berr_nw || steps) {
        if (!h->solved) return QDMF_ERR_NOT_FACTORISED;
        const size_t units = ns * (size_t)h->last_nrhs;
        std::vector<double> bu(4 * units);
        if (hipMemcpy(bu.data(), h->stat_berr, sizeof(double) * bu.size(), hipMemcpyDeviceToHost) != hipSuccess)
            return QDMF_ERR_HIP;
        if (berr_nw)
            for (size_t u = 0; u < units; ++u) berr_nw[u] = bu[4 * u];
        if (steps && hipMemcpy(steps, h->stat_steps, sizeof(int32_t) * units, hipMemcpyDeviceToHost) != hipSuccess)
            return QDMF_ERR_HIP;
    }
    return 0;
}

int qdmf_solve(qdmf_handle h, int32_t nrhs, const double* r7_dev, const double* r1_dev, double* dx_dev,
               double* dy_dev) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->factorised) return QDMF_ERR_NOT_FACTORISED;
    if (nrhs <= 0 || (!r1_dev && h->P.m > 0) || (!dx_dev && h->P.n > 0) || (!dy_dev && h->P.m > 0))
        return QDMF_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    if (h->P.N == 0) {  // an empty system: empty solution, zero backward error
        h->last_nrhs = nrhs;
        h->solved = true;
        return 0;
    }
    if ((rc = ensure_solve(h, nrhs))) return rc;
    enqueue_solve(h, r7_dev, r1_dev, dx_dev, dy_dev);
    if (hipGetLastError() != hipSuccess) return QDMF_ERR_HIP;
    h->last_nrhs = nrhs;
    h->solved = true;
    return 0;
}

int qdmf_solve_noalloc(qdmf_handle h, int32_t nrhs, const double* r7_dev, const double* r1_dev, double* dx_dev,
                       double* dy_dev) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->factorised) return QDMF_ERR_NOT_FACTORISED;
    if (nrhs <= 0 || (!r1_dev && h->P.m > 0) || (!dx_dev && h->P.n > 0) || (!dy_dev && h->P.m > 0))
        return QDMF_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    if (h->P.N == 0) {
        h->last_nrhs = nrhs;
        h->solved = true;
        return 0;
    }
    void* base = scratch_addr(h->device);
    if (!base) {
        h->msg = "qdmf_solve_noalloc: no work space on this device";
        return QDMF_ERR_HIP;
    }
    const bool krylov = krylov_refine(h);
    DevSolve S{};
    DevGmres G{};
    double *V = nullptr, *Z = nullptr, *W = nullptr;
    Carve c;
    layout_solve(h, nrhs, c, S);
    if (krylov) layout_gmres(h, nrhs, c, V, Z, W, G);
    if (c.off > (int64_t)QDMF_NOALLOC_SCRATCH_BYTES) {
        h->msg = "qdmf_solve_noalloc: the work space needs " + std::to_string(c.off) + " bytes, above the " +
                 std::to_string((int64_t)QDMF_NOALLOC_SCRATCH_BYTES) + " of QDMF_NOALLOC_SCRATCH_BYTES";
        return QDMF_ERR_OOM;
    }
    c.base = (char*)base;
    c.off = 0;
    layout_solve(h, nrhs, c, S);
    if (krylov) layout_gmres(h, nrhs, c, V, Z, W, G);
    // the enqueue works on the handle's work space members: point them at the fixed array for
    // this call and give the handle's own back afterwards
    const DevSolve S0 = h->S;
    const DevGmres G0 = h->gm;
    double *V0 = h->gm_V, *Z0 = h->gm_Z, *W0 = h->gm_W;
    const int32_t cap0 = h->gm_cap;
    h->S = S;
    h->gm = G;
    h->gm_V = V;
    h->gm_Z = Z;
    h->gm_W = W;
    h->gm_cap = krylov ? nrhs : 0;
    h->nopoll = true;
    enqueue_solve(h, r7_dev, r1_dev, dx_dev, dy_dev);
    h->nopoll = false;
    h->S = S0;
    h->gm = G0;
    h->gm_V = V0;
    h->gm_Z = Z0;
    h->gm_W = W0;
    h->gm_cap = cap0;
    if (hipGetLastError() != hipSuccess) return QDMF_ERR_HIP;
    h->last_nrhs = nrhs;
    h->solved = true;
    return 0;
}

int qdmf_factor_stats(qdmf_handle h, qdmf_factor_info* out) {
    if (!h || !out) return QDMF_ERR_INVALID_ARG;
    if (!h->factorised) return QDMF_ERR_NOT_FACTORISED;
    if (set_device(h)) return QDMF_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    if (h->P.N == 0) {  // an empty system: no pivots
        *out = qdmf_factor_info{};
        return 0;
    }
    DevStats st;
    DevScalars sc;
    if (hipMemcpy(&st, h->D.st, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess) return QDMF_ERR_HIP;
    if (hipMemcpy(&sc, h->D.sc, sizeof(sc), hipMemcpyDeviceToHost) != hipSuccess) return QDMF_ERR_HIP;
    out->nneg = st.nneg;
    out->npos = st.npos;
    out->nzero = st.nzero;
    out->n2x2 = st.n2x2;
    out->nlift = st.nlift;
    out->nprop3 = st.nprop3;
    out->nsign = st.nsign;
    out->nzskip = st.nzskip;
    out->max_edyn = st.max_edyn;
    out->knorm = sc.knorm;
    out->nredo_fp64 = 0;
    if (h->last_prec == QDMF_MIXED &&
        hipMemcpy(&out->nredo_fp64, h->D.redo + h->P.nsys, sizeof(int32_t), hipMemcpyDeviceToHost) != hipSuccess)
        return QDMF_ERR_HIP;
    int status = 0;
    if (st.bad_theta) status = QDMF_ERR_INVALID_ARG;
    else if (st.large_reg) status = QDMF_WARN_LARGE_REG;
    else if (h->P.mode == QDMF_AS ? (st.nneg != h->P.n || st.npos != h->P.m) : (st.npos != h->P.m))
        status = QDMF_WARN_INERTIA;
    else if (st.nprop3 || st.nsign) status = QDMF_WARN_DYN_REG;
    out->status = status;
    return status;
}

int qdmf_solve_stats(qdmf_handle h, qdmf_solve_info* out, double* berr_nw_per_rhs, int32_t* steps_per_rhs) {
    if (!h || !out) return QDMF_ERR_INVALID_ARG;
    if (!h->solved) return QDMF_ERR_NOT_FACTORISED;
    if (set_device(h)) return QDMF_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    if (h->P.N == 0) {  // an empty system
        *out = qdmf_solve_info{};
        out->nrhs = h->last_nrhs;
        for (int32_t r = 0; r < h->last_nrhs; ++r) {
            if (berr_nw_per_rhs) berr_nw_per_rhs[r] = 0.0;
            if (steps_per_rhs) steps_per_rhs[r] = 0;
        }
        return 0;
    }
    const int32_t nr = h->last_nrhs, ns = h->P.nsys;
    std::vector<double> bu(4 * (size_t)nr * ns), be(4 * (size_t)nr, 0.0);
    std::vector<int32_t> su((size_t)nr * ns), steps(nr, 0);
    if (hipMemcpy(bu.data(), h->stat_berr, sizeof(double) * bu.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return QDMF_ERR_HIP;
    if (hipMemcpy(su.data(), h->stat_steps, sizeof(int32_t) * su.size(), hipMemcpyDeviceToHost) != hipSuccess)
        return QDMF_ERR_HIP;
    for (int32_t r = 0; r < nr; ++r)  // worst system per rhs
        for (int32_t q = 0; q < ns; ++q) {
            const size_t u = (size_t)r * ns + q;
            for (int v = 0; v < 3; ++v) be[4 * r + v] = std::max(be[4 * r + v], bu[4 * u + v]);
            steps[r] = std::max(steps[r], su[u]);
        }
    const bool mixed = h->last_prec == QDMF_MIXED;
    const double target = mixed ? h->opt.target_berr_mixed : h->opt.target_berr;
    out->nrhs = nr;
    out->max_steps = 0;
    out->berr_nw = 0;
    out->berr_cw = 0;
    out->berr_nw_initial = 0;
    for (int32_t r = 0; r < nr; ++r) {
        out->max_steps = std::max(out->max_steps, steps[r]);
        out->berr_nw = std::max(out->berr_nw, be[4 * r]);
        out->berr_cw = std::max(out->berr_cw, be[4 * r + 1]);
        out->berr_nw_initial = std::max(out->berr_nw_initial, be[4 * r + 2]);
        if (berr_nw_per_rhs) berr_nw_per_rhs[r] = be[4 * r];
        if (steps_per_rhs) steps_per_rhs[r] = steps[r];
    }
    out->status = out->berr_nw > target ? QDMF_WARN_NOT_CONVERGED : 0;
    return out->status;
}

int qdmf_export_d(qdmf_handle h, int32_t* pivot_order, double* d, double* doff, int8_t* ptype,
                  double* edyn) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->factorised) return QDMF_ERR_NOT_FACTORISED;
    if (set_device(h)) return QDMF_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    const Plan& P = h->P;
    const size_t N = (size_t)P.N;
    if (N == 0) return 0;
    if (d && hipMemcpy(d, h->D.dval, 8 * N, hipMemcpyDeviceToHost) != hipSuccess) return QDMF_ERR_HIP;
    if (doff && hipMemcpy(doff, h->D.doff, 8 * N, hipMemcpyDeviceToHost) != hipSuccess) return QDMF_ERR_HIP;
    if (ptype && hipMemcpy(ptype, h->D.ptype, N, hipMemcpyDeviceToHost) != hipSuccess) return QDMF_ERR_HIP;
    if (edyn && hipMemcpy(edyn, h->D.edyn, 8 * N, hipMemcpyDeviceToHost) != hipSuccess) return QDMF_ERR_HIP;
    if (pivot_order) {
        std::vector<int32_t> lp(N);
        if (hipMemcpy(lp.data(), h->D.lperm, 4 * N, hipMemcpyDeviceToHost) != hipSuccess) return QDMF_ERR_HIP;
        for (int32_t s = 0; s < P.ns; ++s)
            for (int32_t k = P.sn_ptr[s]; k < P.sn_ptr[s + 1]; ++k) pivot_order[k] = P.perm[P.sn_ptr[s] + lp[k]];
    }
    return 0;
}

int qdmf_export_flags(qdmf_handle h, uint8_t* flags) {
    if (!h || !flags) return QDMF_ERR_INVALID_ARG;
    if (!h->factorised) return QDMF_ERR_NOT_FACTORISED;
    if (set_device(h)) return QDMF_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    const size_t N = (size_t)h->P.N;
    if (N && hipMemcpy(flags, h->D.pflag, N, hipMemcpyDeviceToHost) != hipSuccess) return QDMF_ERR_HIP;
    return 0;
}

int qdmf_export_front(qdmf_handle h, int32_t s, double* panel, int32_t* rows) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->factorised) return QDMF_ERR_NOT_FACTORISED;
    const Plan& P = h->P;
    if (s < 0 || s >= P.ns) return QDMF_ERR_INVALID_ARG;
    if (set_device(h)) return QDMF_ERR_HIP;
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    const int32_t f = P.sn_f[s], p = P.sn_p[s], c0 = P.sn_ptr[s];
    if (panel) {
        if (hipMemcpy(panel, h->D.front + P.sn_off[s], sizeof(double) * (size_t)f * p, hipMemcpyDeviceToHost) !=
            hipSuccess)
            return QDMF_ERR_HIP;
    }
    if (rows) {
        std::vector<int32_t> lp(p > 0 ? p : 1);
        if (p > 0 && hipMemcpy(lp.data(), h->D.lperm + c0, 4 * (size_t)p, hipMemcpyDeviceToHost) != hipSuccess)
            return QDMF_ERR_HIP;
        for (int32_t k = 0; k < p; ++k) rows[k] = P.perm[c0 + lp[k]];
        for (int32_t k = p; k < f; ++k) rows[k] = P.perm[P.rows[P.sn_rowptr[s] + k]];
    }
    return 0;
}

namespace {

int graph_capture_impl(qdmf_handle h, const double* theta_dev, double rho, double delta, const double* rho_dev,
                       const double* delta_dev, int32_t prec, int32_t nsolves, int32_t nrhs, const double* r7_dev,
                       const double* r1_dev, double* dx_dev, double* dy_dev) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    if (!h->analysed) return QDMF_ERR_NOT_ANALYSED;
    if (!h->have_matrix || (h->P.has_q && !h->have_hessian)) return QDMF_ERR_NO_MATRIX;
    if (h->host_only || !h->stream || nsolves < 0 || nrhs <= 0 || h->P.N == 0 || (!theta_dev && h->P.n > 0) ||
        (prec != QDMF_FP64 && prec != QDMF_MIXED) || !(rho >= 0) || !(delta >= 0))
        return QDMF_ERR_INVALID_ARG;
    if (set_device(h)) return QDMF_ERR_HIP;
    int rc = ensure_solve(h, nrhs);
    if (rc) return rc;
    // every buffer the captured work uses exists before the capture starts
    if (prec == QDMF_MIXED && h->fp32_fronts && h->opt.max_refine_mixed > 0 && (rc = ensure_gmres(h))) return rc;
    destroy_graph(h);
    const int32_t units = nrhs * h->P.nsys;
    if (h->opt.graph_poll && h->poll_cap < units) {
        if (h->poll_host) (void)hipHostFree(h->poll_host);
        h->poll_host = nullptr;
        h->poll_cap = 0;
        if (hipHostMalloc((void**)&h->poll_host, sizeof(int32_t) * std::max(units, 1), hipHostMallocDefault) !=
            hipSuccess) {
            h->poll_host = nullptr;
            return QDMF_ERR_OOM;
        }
        h->poll_cap = std::max(units, 1);
    }
    if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
    if (hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return QDMF_ERR_HIP;
    h->cut_capture = h->opt.graph_poll != 0;
    h->capture_failed = false;
    h->cur_flag = nullptr;
    h->cur_nflag = 0;
    h->skip_pending.clear();
    // the enqueue code reads the precision of the factorisation it follows; nothing has run
    // yet, so the handle's own state is restored after the capture
    const int32_t prec_before = h->last_prec;
    h->last_prec = prec;
    h->capturing = true;
    enqueue_factorise(h, theta_dev, rho, delta, rho_dev, delta_dev, prec);
    for (int32_t q = 0; q < nsolves; ++q) enqueue_solve(h, r7_dev, r1_dev, dx_dev, dy_dev);
    seg_close(h);
    h->capturing = false;
    h->cut_capture = false;
    h->last_prec = prec_before;
    for (size_t q = 0; q < h->segs.size(); ++q) h->segs[q].skip_to = q + 1;
    for (const auto& sk : h->skip_pending) h->segs[(size_t)sk.first].skip_to = (size_t)sk.second;
    h->skip_pending.clear();
    if (h->capture_failed) {
        destroy_graph(h);
        return QDMF_ERR_HIP;
    }
    h->graph_prec = prec;
    h->graph_nrhs = nrhs;
    h->graph_nsolves = nsolves;
    return 0;
}

}  // namespace

int qdmf_graph_capture(qdmf_handle h, const double* theta_dev, double rho, double delta, int32_t prec,
                       int32_t nsolves, int32_t nrhs, const double* r7_dev, const double* r1_dev, double* dx_dev,
                       double* dy_dev) {
    return graph_capture_impl(h, theta_dev, rho, delta, nullptr, nullptr, prec, nsolves, nrhs, r7_dev, r1_dev, dx_dev,
                              dy_dev);
}

int qdmf_batch_graph_capture(qdmf_handle h, const double* theta_dev, const double* rho_dev,
                             const double* delta_dev, int32_t prec, int32_t nsolves, int32_t nrhs,
                             const double* r7_dev, const double* r1_dev, double* dx_dev, double* dy_dev) {
    if (!rho_dev || !delta_dev) return QDMF_ERR_INVALID_ARG;
    return graph_capture_impl(h, theta_dev, 0.0, 0.0, rho_dev, delta_dev, prec, nsolves, nrhs, r7_dev, r1_dev, dx_dev,
                              dy_dev);
}

int qdmf_graph_launch(qdmf_handle h) {
    if (!h || h->segs.empty()) return QDMF_ERR_INVALID_ARG;
    if (set_device(h)) return QDMF_ERR_HIP;
    for (size_t q = 0; q < h->segs.size();) {
        const qdmf_ctx::GraphSeg& g = h->segs[q];
        if (g.flag) {  // a decision point: read its flags, as an eager solve does
            if (g.nflag > h->poll_cap ||
                hipMemcpyAsync(h->poll_host, g.flag, sizeof(int32_t) * g.nflag, hipMemcpyDeviceToHost, h->stream) !=
                    hipSuccess ||
                hipStreamSynchronize(h->stream) != hipSuccess)
                return QDMF_ERR_HIP;
            bool any = false;
            for (int32_t u = 0; u < g.nflag; ++u) any = any || h->poll_host[u] != 0;
            if (!any) {
                q = g.skip_to;
                continue;
            }
        }
        if (g.x && hipGraphLaunch(g.x, h->stream) != hipSuccess) return QDMF_ERR_HIP;
        ++q;
    }
    // the handle now holds the graph's factorisation and, with solves, their statistics
    h->last_prec = h->graph_prec;
    h->factorised = true;
    h->last_nrhs = h->graph_nrhs;
    h->solved = h->graph_nsolves > 0;
    h->stat_berr = h->S.berr;
    h->stat_steps = h->S.steps;
    return 0;
}

int qdmf_profile_kind(qdmf_handle h, int32_t kind) {
    if (!h || kind < -1 || kind > QDMF_K_SYRK128) return QDMF_ERR_INVALID_ARG;
    h->prof_kind = kind;
    return 0;
}

int qdmf_profile_read(qdmf_handle h, int64_t* launches, double* total_ms, double* flops, double* bytes) {
    if (!h) return QDMF_ERR_INVALID_ARG;
    double ms = 0.0;
    if (h->ev_used) {
        if (set_device(h)) return QDMF_ERR_HIP;
        if (hipStreamSynchronize(h->stream) != hipSuccess) return QDMF_ERR_HIP;
        for (size_t q = 0; q + 1 < h->ev_used; q += 2) {
            float t = 0.f;
            if (hipEventElapsedTime(&t, h->ev_pool[q], h->ev_pool[q + 1]) != hipSuccess) return QDMF_ERR_HIP;
            ms += t;
        }
    }
    if (launches) *launches = (int64_t)(h->ev_used / 2);
    if (total_ms) *total_ms = ms;
    if (flops) *flops = h->prof_flops;
    if (bytes) *bytes = h->prof_bytes;
    h->ev_used = 0;
    h->prof_flops = h->prof_bytes = 0;
    return 0;
}

void qdmf_ipm_default_options(qdmf_ipm_options* o) {
    if (!o) return;
    o->tau = 1e-8;
    o->rho = 1e-10;
    o->delta = 1e-10;
    o->max_iter = 100;
    o->correctors = 0;
    o->kmax = 6;
    o->alpha_f = 0.025;
    o->prec = QDMF_FP64;
}

int qdmf_ipm_solve(qdmf_handle h, const double* b_dev, const double* c_dev, const double* l_dev,
                   const double* u_dev, double* x_dev, double* y_dev, double* zl_dev, double* zu_dev,
                   const qdmf_ipm_options* opt_in, qdmf_ipm_info* info, double* history) {
    // readings shared with the reference implementation the tests compare against
    constexpr double STEP_FACTOR = 0.995, ALPHA_PLUS = 0.1, BETA_MIN = 0.1, BETA_MAX = 10.0, ACCEPT_GAIN = 0.01;
    if (!h || !info || !b_dev || !c_dev || !x_dev || !y_dev || !zl_dev || h->host_only) return QDMF_ERR_INVALID_ARG;
    if (!h->analysed || h->P.mode != QDMF_AS || h->P.nsys != 1) return QDMF_ERR_NOT_ANALYSED;
    if (!h->have_matrix || (h->P.has_q && !h->have_hessian)) return QDMF_ERR_NO_MATRIX;
    if (h->P.m == 0 || h->P.n == 0) return QDMF_ERR_INVALID_ARG;
    qdmf_ipm_options opt;
    if (opt_in) opt = *opt_in;
    else qdmf_ipm_default_options(&opt);
    if (opt.max_iter < 0 || opt.correctors < 0 || opt.kmax < 1 || !(opt.tau > 0) || opt.rho < 0 || opt.delta < 0)
        return QDMF_ERR_INVALID_ARG;
    int rc = set_device(h);
    if (rc) return rc;
    const int n = h->P.n, m = h->P.m;
    hipStream_t st = h->stream;
    // Section 4.7: (1 + k)(1 + f/2) E_s ~ E_f alpha_F, E_s = 2 nnz(L), E_f = factorisation flops
    int k = opt.correctors;
    if (k == 0) {
        const double es = 2.0 * (double)h->P.nnz_l, f = h->opt.max_refine;
        k = (int)std::floor(opt.alpha_f * h->P.flops_fact / ((1.0 + f / 2.0) * es) - 1.0);
        k = std::max(1, std::min(opt.kmax, k));
    }
    // work space
    std::vector<void*> mem;
    auto alloc = [&](double** p, int64_t len) {
        *p = nullptr;
        if (hipMalloc((void**)p, sizeof(double) * (size_t)std::max<int64_t>(1, len)) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        mem.push_back(*p);
        return true;
    };
    auto alloc_vec = [&](IpmVec& v) {
        return alloc(&v.x, n) && alloc(&v.xl, n) && alloc(&v.xu, n) && alloc(&v.y, m) && alloc(&v.zl, n) &&
               alloc(&v.zu, n);
    };
    IpmVec pt{x_dev, nullptr, nullptr, y_dev, zl_dev, zu_dev}, da{}, db{}, dc{};
    double *theta, *r1, *r2, *r3, *r4, *r5, *r6, *r7, *zm, *part, *out;
    const int64_t nparts = IPM_PART * (int64_t)ipm_blocks(std::max(n, m));
    bool ok = alloc(&pt.xl, n) && alloc(&pt.xu, n) && (zu_dev || alloc(&pt.zu, n)) && alloc_vec(da) &&
              alloc_vec(db) && alloc_vec(dc) && alloc(&theta, n) && alloc(&r1, m) && alloc(&r2, n) &&
              alloc(&r3, n) && alloc(&r4, n) && alloc(&r5, n) && alloc(&r6, n) && alloc(&r7, n) && alloc(&zm, m) &&
              alloc(&part, nparts) && alloc(&out, 16);
    auto release = [&]() {
        for (void* p : mem) (void)hipFree(p);
    };
    if (!ok) {
        release();
        return QDMF_ERR_OOM;
    }
    double sc[16];
    auto read = [&](int cnt) {
        return hipMemcpyAsync(sc, out, sizeof(double) * cnt, hipMemcpyDeviceToHost, st) == hipSuccess &&
               hipStreamSynchronize(st) == hipSuccess;
    };
    const auto t0 = std::chrono::steady_clock::now();
    ipm_start(l_dev, u_dev, pt, n, m, part, out, st);
    ipm_fill(zm, 0.0, m, st);
    if (!read(2)) {
        release();
        return QDMF_ERR_HIP;
    }
    if (sc[0] != 0.0) {
        release();
        h->msg = "qdmf_ipm_solve: every l must be finite and every finite u above its l";
        return QDMF_ERR_INVALID_ARG;
    }
    const double ncomp = (double)n + sc[1];  // complementarity pairs
    qdmf_ipm_info res{};
    res.status = QDMF_WARN_NOT_CONVERGED;
    res.correctors = k;
    int it = 0;
    rc = 0;
    for (;; ++it) {
        ipm_resid(h->D, pt, b_dev, c_dev, l_dev, u_dev, r1, r2, r3, r4, part, out, st);
        if (!read(14)) {
            rc = QDMF_ERR_HIP;
            break;
        }
        const double pinf = std::max(sc[0], std::max(sc[7], sc[8])), dinf = sc[1];
        const double half_xqx = 0.5 * sc[13];  // 0 for a linear program
        const double fp = sc[2] + half_xqx, fd = sc[3] + sc[9] - sc[10] - half_xqx, comp = sc[4];
        const double pscale = std::max(sc[5], std::max(sc[11], sc[12])), cmax = sc[6];
        res.pinf = pinf;
        res.dinf = dinf;
        res.primal_obj = fp;
        res.dual_obj = fd;
        res.mu = ncomp > 0 ? comp / ncomp : 0.0;
        // Section 3.1, without scaling
        if (pinf <= opt.tau * (1.0 + pscale) && dinf <= opt.tau * (1.0 + cmax) &&
            std::fabs(fp - fd) <= opt.tau * (1.0 + 0.5 * std::fabs(fp + fd))) {
            res.status = 0;
            break;
        }
        if (it >= opt.max_iter) break;
        const double mu = res.mu;
        ipm_theta(pt, u_dev, theta, n, st);
        if ((rc = qdmf_factorise(h, theta, opt.rho, opt.delta, opt.prec)) < 0) break;
        // predictor (sigma = 0)
        ipm_rhs(0, pt, da, u_dev, r2, r3, r4, 0.0, 0.0, 0.0, 0.0, 0.0, r5, r6, r7, n, st);
        if ((rc = qdmf_solve(h, 1, r7, r1, da.x, da.y)) < 0) break;
        ipm_recover(pt, da, u_dev, r2, r3, r5, r6, n, st);
        ipm_step(pt, da, u_dev, part, out, n, st);
        if (!read(2)) {
            rc = QDMF_ERR_HIP;
            break;
        }
        double ap = -sc[0], ad = -sc[1];
        ipm_comp(pt, da, u_dev, ap, ad, part, out, n, st);
        if (!read(1)) {
            rc = QDMF_ERR_HIP;
            break;
        }
        const double mu_aff = sc[0] / ncomp, sigma = (mu_aff / mu) * (mu_aff / mu) * (mu_aff / mu), smu = sigma * mu;
        // correctors: r1 = r2 = r3 = r4 = 0; r5, r6 move the products at the trial point into
        // the band [BETA_MIN, BETA_MAX] * sigma * mu
        IpmVec d = da, nd = db;
        int used = 0;
        for (int j = 0; j < k; ++j) {
            const double tp = std::min(1.0, ap + ALPHA_PLUS), td = std::min(1.0, ad + ALPHA_PLUS);
            ipm_rhs(1, pt, d, u_dev, nullptr, nullptr, nullptr, smu, tp, td, BETA_MIN, BETA_MAX, r5, r6, r7, n, st);
            if ((rc = qdmf_solve(h, 1, r7, zm, dc.x, dc.y)) < 0) break;
            ipm_recover(pt, dc, u_dev, nullptr, nullptr, r5, r6, n, st);
            ipm_add(d, dc, nd, n, m, st);
            ipm_step(pt, nd, u_dev, part, out, n, st);
            if (!read(2)) {
                rc = QDMF_ERR_HIP;
                break;
            }
            const double nap = -sc[0], nad = -sc[1];
            if (j > 0 && nap + nad < (1.0 + ACCEPT_GAIN) * (ap + ad)) break;
            std::swap(d, nd);  // the accepted direction; the old one's buffers become the spares
            ap = nap;
            ad = nad;
            ++used;
        }
        if (rc < 0) break;
        if (history && it < opt.max_iter) {
            history[4 * it] = mu;
            history[4 * it + 1] = ap;
            history[4 * it + 2] = ad;
            history[4 * it + 3] = used;
        }
        ipm_update(pt, d, STEP_FACTOR * ap, STEP_FACTOR * ad, n, m, st);
    }
    if (hipStreamSynchronize(st) != hipSuccess && rc == 0) rc = QDMF_ERR_HIP;
    res.iters = it;
    res.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    release();
    *info = res;
    return rc < 0 ? rc : res.status;
}

int qdmf_choose_mode(qdmf_handle h, int32_t m, int32_t n, const int64_t* colptr, const int32_t* rowidx,
                     qdmf_mode_choice* out) {
    if (!h || !out) return QDMF_ERR_INVALID_ARG;
    if (h->opt.ordering == QDMF_ORDER_USER || h->opt.ordering == QDMF_ORDER_GRID_ND) {
        h->msg = "qdmf_choose_mode needs an ordering computed from the pattern (AMD, ND or AUTO)";
        return QDMF_ERR_INVALID_ARG;
    }
    qdmf_mode_choice c{};
    c.nnz_ne_pattern = -1;
    c.nnz_l_ne = -1;
    c.flops_ne = -1.0;
    AnalyseOptions ao;
    ao.ordering = h->opt.ordering;
    ao.amalgamate = h->opt.amalgamate;
    ao.small_front = h->opt.small_front;
    ao.split_solve_front = h->opt.split_solve_front;
    ao.syrk_group_front = h->opt.syrk_group_front;
    ao.syrk_group = h->opt.syrk_group;
    ao.syrk_tile_front = h->opt.syrk_tile_front;
    ao.lookahead_front = h->opt.lookahead_front;
    ao.f_mix = h->opt.f_mix;
    {  // the augmented system first
        Plan Pa;
        const int rc = build_plan(m, n, colptr, rowidx, QDMF_AS, ao, Pa, h->msg);
        if (rc) return rc;
        c.nnz_l_as = Pa.nnz_l;
        c.flops_as = Pa.flops_fact;
    }
    const int64_t dense_min = std::max<int64_t>(64, ((int64_t)m + 9) / 10);
    for (int32_t j = 0; j < n; ++j)
        if (colptr[j + 1] - colptr[j] >= dense_min) ++c.ndense;
    c.mode = QDMF_AS;
    if (c.ndense > 0) {
        c.ne_abandoned = 1;
    } else {
        c.nnz_ne_pattern = ne_pattern_count(m, n, colptr, rowidx, c.nnz_l_as);
        if (c.nnz_ne_pattern > c.nnz_l_as) {
            c.ne_abandoned = 1;
        } else {
            Plan Pn;
            const int rc = build_plan(m, n, colptr, rowidx, QDMF_NE, ao, Pn, h->msg);
            if (rc) return rc;
            c.nnz_l_ne = Pn.nnz_l;
            c.flops_ne = Pn.flops_fact;
            if (c.flops_ne <= c.flops_as) c.mode = QDMF_NE;
        }
    }
    *out = c;
    return 0;
}

void qdmf_destroy(qdmf_handle h) {
    if (!h) return;
    if (!h->host_only) {
        (void)hipSetDevice(h->device);
        (void)hipStreamSynchronize(h->stream);
    }
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->ev_win) (void)hipEventDestroy(h->ev_win);
    if (h->ev_s2) (void)hipEventDestroy(h->ev_s2);
    if (h->stream2) (void)hipStreamDestroy(h->stream2);
    if (h->act_host) (void)hipHostFree(h->act_host);
    if (h->gm_act_host) (void)hipHostFree(h->gm_act_host);
    if (h->shift_host) (void)hipHostFree(h->shift_host);
    if (h->poll_host) (void)hipHostFree(h->poll_host);
    destroy_graph(h);
    free_list(h->solve_allocs);
    free_list(h->plan_allocs);
    delete h;
}

const char* qdmf_status_string(int code) {
    switch (code) {
        case QDMF_OK: return "ok";
        case QDMF_ERR_INVALID_ARG: return "invalid argument";
        case QDMF_ERR_HIP: return "HIP runtime error";
        case QDMF_ERR_OOM: return "out of memory (plan above cap or allocation failed)";
        case QDMF_ERR_INDEX_OVERFLOW: return "32-bit index overflow";
        case QDMF_ERR_NOT_ANALYSED: return "not analysed";
        case QDMF_ERR_NOT_FACTORISED: return "not factorised";
        case QDMF_ERR_NO_MATRIX: return "matrix values not set";
        case QDMF_ERR_UNSUPPORTED: return "unsupported problem shape";
        case QDMF_WARN_DYN_REG: return "dynamic regularisation applied";
        case QDMF_WARN_INERTIA: return "inertia differs from the quasi-definite inertia";
        case QDMF_WARN_NOT_CONVERGED: return "refinement did not reach the target backward error";
        case QDMF_WARN_LARGE_REG: return "regularisation larger than tau_big * ||K||_1";
        default: return "unknown status";
    }
}

// Last error message of a handle (diagnostics).
const char* qdmf_last_message(qdmf_handle h) { return h ? h->msg.c_str() : ""; }

}  // extern "C"
