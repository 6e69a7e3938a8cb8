// Device-side data of one analysed system and the host wrappers that launch the kernels.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace qdmf {

// Per-position pivot flags written by the pivot kernels.
enum : uint8_t { PF_LIFT = 1, PF_PROP3 = 2, PF_SIGN = 4 };

// Scalars shared by the kernels of one factorisation (device memory).
struct DevScalars {
    double knorm;      // ||K_static||_1
    double rho, delta;
    int32_t bad_theta; // set if some Theta_j is not positive and finite
    int32_t pad;
};

// Factorisation statistics (device memory, reduced at the end of a factorisation).
struct DevStats {
    int64_t nneg, npos, nzero, n2x2, nlift, nprop3, nsign, nzskip;
    double max_edyn;
    int32_t large_reg, bad_theta;
};

struct PivotParams {
    double alpha, eps_lift, tau_big;
    int32_t presort;
    int32_t mixed;  // 1: FP32 Schur updates on fronts with f >= f_mix
    int32_t f_mix;
    int32_t mixed_check;  // which broken-down mixed factors are redone in FP64 (qdmf_options)
};

struct DevPlan {
    int32_t N, n, m, mode, ns;
    int64_t ub_total;
    // supernodes
    const int32_t* sn_ptr;
    const int32_t* sn_parent;
    const int32_t* sn_f;
    const int32_t* sn_p;
    const int32_t* sn_ld;
    const int64_t* sn_off;
    const int64_t* sn_rowptr;
    const int32_t* rows;
    const int32_t* ch_ptr;
    const int32_t* ch;
    const int64_t* rel_ptr;
    const int32_t* rel;
    const int64_t* ub_off;
    const int64_t* yoff;      // per supernode: rows in the solve work space (big supernodes)
    const int64_t* inv_off;   // per supernode: inverses of its diagonal blocks in linv, or -1
    double* linv;
    const int64_t* fg_ptr;    // forward-solve gather list per front row
    const int64_t* fg_src;
    // K entries
    const int64_t* kcol_ptr;
    const int32_t* kloc;      // row position of each entry in its front
    const int32_t* kcl;       // column position of each entry in its front
    const int32_t* asm_child; // per large-front column task: (child, child CB column) pairs
    const int32_t* asm_col;
    const int64_t* ksrc;      // AS
    const int64_t* kpair_ptr; // NE
    const int32_t* kpair;
    const int64_t* krs_ptr;   // NE
    const int32_t* krs_ent;
    const int32_t* krs_other;
    const int8_t* primal_new;
    const int32_t* perm;      // new -> old
    // AS: columns of A with more than LONG_COL entries, and per column its index among them or -1
    int32_t nlong;
    const int32_t* long_col;
    const int32_t* long_of;
    // A
    const int64_t* acp;
    const int32_t* ari;
    const int64_t* arp;
    const int32_t* are;
    const int32_t* acol;
    // quadratic programs (AS): has_q, the full symmetric pattern of Q (CSC) with the index of
    // each value in qval (the lower triangle as given), the diagonal's index per column (-1:
    // none), and per column the sum of |Q_kj| over k != j
    int32_t has_q;
    const int64_t* qfcp;
    const int32_t* qfri;
    const int64_t* qfsrc;
    const int64_t* qdiag;
    double* qval;
    double* qoff;
    // numeric state (owned by the handle)
    double* front;
    double* kval;
    double* aval;
    double* colabs;   // sum_i |A_ij|
    double* rowabs;   // sum_j |A_ij|
    double* dinv;     // AS: 1/Theta; NE: theta~
    double* rowsum;   // row 1-norms of K_static (original numbering)
    double* dval;
    double* doff;
    int8_t* ptype;
    double* edyn;
    uint8_t* pflag;
    int32_t* zskip;
    int32_t* lperm;   // by position: pre-pivot local position now pivoted there
    int32_t* lpinv;   // inverse: c0 + pre-pivot local position -> post-pivot local position
    DevScalars* sc;
    DevStats* st;
    // systems (one unless a batch): per-system ||K_static||_1 and static shifts, and maps
    int32_t nsys;
    const int32_t* sys_col;      // per column of A
    const int32_t* sys_old;      // per K index, original numbering
    const int32_t* sys_new;      // per K index, elimination order
    const int64_t* sys_rng;      // per system: [a0, a1), [b0, b1) in original numbering
    const int64_t* sys_piv_ptr;  // per system: pivot positions
    const int32_t* sys_piv;
    const int32_t* sn_sys;       // per supernode: its system
    // Mixed precision: per system 1 if its factorisation is redone in FP64 (the FP32 Schur
    // updates broke down), then the number of such systems (nsys + 1 entries).  The factor
    // kernels launched with gate = redo skip the supernodes of the systems marked 0; gate is
    // NULL otherwise.
    int32_t* redo;
    const int32_t* gate;
    double* knorm_sys;
    double* rho_sys;
    double* delta_sys;
    int64_t* inertia_sys;        // per system: negative, positive, zero pivots
};

// ---- factorisation
// rho_sys/delta_sys: per-system shifts (device, nsys each) or NULL to use rho, delta for all
void launch_theta(const DevPlan& D, const double* theta, double rho, double delta, const double* rho_sys,
                  const double* delta_sys, hipStream_t s);
void launch_values_n(const DevPlan& D, int64_t knnz, hipStream_t s);
void launch_knorm(const DevPlan& D, hipStream_t s);
void launch_factor_step(const DevPlan& D, const Launch& L, const Task* tasks_dev,
                        const PivotParams& pp, hipStream_t s);
// part: factor_stats_blocks(N) x 10 doubles of device scratch
int factor_stats_blocks(int64_t N);
void launch_factor_stats(const DevPlan& D, const PivotParams& pp, double* part, hipStream_t s);
// Marks in D.redo the systems whose mixed-precision factor broke down and counts them in
// D.redo[nsys]; max_piv is the largest pivot count of one system.
void launch_mixed_check(const DevPlan& D, const PivotParams& pp, int64_t max_piv, hipStream_t s);
void launch_matrix_norms(const DevPlan& D, hipStream_t s);
void launch_hessian_norms(const DevPlan& D, hipStream_t s);

// ---- solve
// Work state of one solve call (device memory owned by the handle).
struct DevSolve {
    int32_t nrhs;
    double* b;      // system right-hand side, original numbering, N x nrhs
    double* x;      // solution, N x nrhs
    double* xbak;
    double* r;      // residual / correction right-hand side, N x nrhs
    double* d;      // correction, N x nrhs
    double* xw;     // permuted work vector, N x nrhs
    double* ub;     // contribution buffers, ub_total x nrhs
    double* part;   // per-block partial maxima: |r|, |x|, |b| (3 x nblk x nrhs), then componentwise ratios (nblk x nrhs)
    int32_t nblk;
    // refinement state per unit u = rhs * nsys + system
    double* berr;     // per unit: [nw, cw, nw_initial, unused]
    int32_t* active;  // per unit: refinement continues
    int32_t* steps;   // per unit
    int32_t* ract;    // per rhs: some system of it still refines (gates the solve kernels)
    double* Y;        // big-supernode work space, ytot x nrhs
    int64_t ytot;
    double* P;        // partial sums of the big backward solves: ppart_max x SOLVE_BLOCK x nrhs
    double* lsum;     // AS: per long column and rhs, sum_i A_ij x_i and sum_i |A_ij||x_i| (2 x nlong x nrhs)
};

void launch_rhs(const DevPlan& D, const DevSolve& S, const double* r7, const double* r1, hipStream_t s);
// Solve building blocks: src (original numbering) -> permuted work vector; one tree level of
// the forward (leaves first) or backward (roots first) pass, one workgroup per supernode;
// work vector -> dst.  rhs with active[r] == 0 are skipped (active may be NULL).
void launch_permute(const DevPlan& D, const DevSolve& S, const double* src, const int32_t* active,
                    hipStream_t s);
void launch_unpermute(const DevPlan& D, const DevSolve& S, double* dst, const int32_t* active, hipStream_t s);
void launch_solve_level(bool forward, const DevPlan& D, const DevSolve& S, const int32_t* lvl_sn_dev,
                        int64_t base, unsigned count, int32_t maxf, int32_t maxp, const int32_t* active,
                        hipStream_t s);
// Inverses of the diagonal blocks used by the one-workgroup solves (after the factorisation).
void launch_inv(const DevPlan& D, const Task* tasks, int64_t ntask, hipStream_t s);
// Interior point driver kernels (ipm.hip).  A point or a direction of the bounded LP
// min c^T x, A x = b, x - x^l = l, x + x^u = u: the six vectors x, x^l, x^u, y, z^l, z^u
// (y of length m, the others n).  Entries of x^u and z^u without a finite upper bound stay 0.
// l == nullptr means l = 0; u == nullptr means u = +inf everywhere.  out: device scalars;
// part: IPM_PART x ipm_blocks(len) doubles of partials.
struct IpmVec {
    double *x, *xl, *xu, *y, *zl, *zu;
};
constexpr int IPM_PART = 16;
int ipm_blocks(int64_t len);
// start point and argument check; out[0] = number of bad bounds, out[1] = number of finite u
void ipm_start(const double* l, const double* u, IpmVec p, int n, int m, double* part, double* out, hipStream_t s);
// r1..r4 and the scalars of the termination test (out[0..12], see ipm.hip)
void ipm_resid(const DevPlan& D, IpmVec p, const double* b, const double* c, const double* l, const double* u,
               double* r1, double* r2, double* r3, double* r4, double* part, double* out, hipStream_t s);
void ipm_theta(IpmVec p, const double* u, double* theta, int n, hipStream_t s);
// mode 0: predictor right-hand sides r5, r6, r7; mode 1: centrality corrector from direction d
void ipm_rhs(int mode, IpmVec p, IpmVec d, const double* u, const double* r2, const double* r3, const double* r4,
             double smu, double tp, double td, double bmin, double bmax, double* r5, double* r6, double* r7, int n,
             hipStream_t s);
// the rest of a direction from its dx (r2 == r3 == nullptr: zero)
void ipm_recover(IpmVec p, IpmVec d, const double* u, const double* r2, const double* r3, const double* r5,
                 const double* r6, int n, hipStream_t s);
void ipm_add(IpmVec a, IpmVec b, IpmVec out, int n, int m, hipStream_t s);
// out[0] = -alpha_p, out[1] = -alpha_d (steps to the boundary, at most 1)
void ipm_step(IpmVec p, IpmVec d, const double* u, double* part, double* out, int n, hipStream_t s);
// out[0] = sum of the complementarity products at p + (ap, ad) d
void ipm_comp(IpmVec p, IpmVec d, const double* u, double ap, double ad, double* part, double* out, int n,
              hipStream_t s);
void ipm_update(IpmVec p, IpmVec d, double sp, double sd, int n, int m, hipStream_t s);
void ipm_fill(double* v, double a, int len, hipStream_t s);
// One launch of the big-supernode solves (kind: SolveKind).
void launch_big_solve(const DevPlan& D, const DevSolve& S, const SolveLaunch& L, const Task* stasks,
                      const int32_t* active, hipStream_t s);
void launch_residual(const DevPlan& D, const DevSolve& S, const double* x, hipStream_t s);
void launch_berr_steps(const DevPlan& D, const DevSolve& S, int32_t phase, double target,
                       int max_steps, hipStream_t s);
void launch_refine_begin(const DevPlan& D, const DevSolve& S, hipStream_t s);
void launch_refine_update(const DevPlan& D, const DevSolve& S, hipStream_t s);
void launch_recover(const DevPlan& D, const DevSolve& S, const double* r7, double* dx, double* dy,
                    hipStream_t s);
void launch_zero(double* p, int64_t n, hipStream_t s);

// ---- Krylov refinement building blocks (N x nrhs blocks, original numbering; act: per rhs,
// skip where 0, or NULL)
// Krylov correction of mixed-precision refinement (device GMRES, right-preconditioned by the
// factor), one Krylov process per refinement unit u = r * nsys + q (U = nrhs * nsys units):
// h1, h2, nrm ((GM_M + 1) x U, unit fastest: the Gram-Schmidt coefficients of both passes and
// squared norms), beta (U), g ((GM_M + 1) per unit), cs, sn (GM_M per unit), R (GM_M x GM_M per
// unit), y (GM_M x U, unit fastest), kr and act (U), ract (nrhs: some unit of the rhs is active).
constexpr int GM_M = 8;
struct DevGmres {
    double *h1, *h2, *nrm, *beta, *g, *cs, *sn, *R, *y;
    int32_t *kr, *act, *ract;
};
void launch_matvec(const DevPlan& D, const double* v, double* out, int nrhs, double* lsum, const int32_t* act,
                   hipStream_t s);
void launch_dots(const DevPlan& D, const double* V, int nv, const double* w, double* out, int nrhs,
                 const int32_t* act, hipStream_t s);
void launch_vcombine(const DevPlan& D, const double* V, int nv, const double* h, double* w, int nrhs, bool subtract,
                     const int32_t* act, const int32_t* nvr, hipStream_t s);
void launch_vscale(const DevPlan& D, const double* src, const double* nrm2, double* dst, int nrhs,
                   const int32_t* act, hipStream_t s);
void launch_gm_start(const DevGmres& G, const int32_t* gate, int nu, hipStream_t s);
void launch_gm_rotate(const DevGmres& G, int j, int nrhs, int nsys, double tol, hipStream_t s);
void launch_gm_gate(const DevGmres& G, int nrhs, int nsys, hipStream_t s);
void launch_gm_solve(const DevGmres& G, int nu, hipStream_t s);

}  // namespace qdmf
