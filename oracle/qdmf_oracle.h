/*
 * Reference (oracle) implementation of the regularised multifrontal LDL^T used by an LP
 * interior point method (Zanetti & Gondzio, arXiv 2508.04370, Sections 3-4).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or calls this
 * code; only the test-suite, the smoke check and the benchmark's CPU-baseline leg do.
 * It shares no source with the GPU library.  Plain loops, FP64, no BLAS, single thread.
 */
#ifndef QDMF_ORACLE_H
#define QDMF_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_NE = 0, ORC_AS = 1 };
/* dynamic regularisation applied to a 1x1 pivot (Sections 4.5-4.6) */
enum { ORC_EF_LIFT = 1, ORC_EF_PROP3 = 2, ORC_EF_SIGN = 4 };

typedef struct {
    int nb;             /* pivot window width (Section 4.4: blocks of 32/64/128 columns)     */
    double alpha;       /* Bunch-Kaufman constant, (1+sqrt(17))/8 (Section 4.5)             */
    double eps_lift;    /* lift parameter "of the order of machine precision" (Section 4.5) */
    int presort;        /* extra swap putting the largest diagonal first (Section 4.5)     */
    int max_refine;     /* refinement steps (Section 4.5)                                   */
    double target_berr; /* stop refinement at this normwise backward error                 */
    double tau_big;     /* "regularisation too large" warning threshold (Section 4.6)      */
} orc_opts;

typedef struct {
    int64_t nneg, npos, nzero;   /* inertia of D                                           */
    int64_t n2x2, nlift, nprop3, nsign, nzskip;
    double max_edyn;             /* max |E_dyn|                                            */
    int large_reg;               /* some |E_dyn| > tau_big * ||K||_1                       */
    int64_t nbkd;                /* Bunch-Kaufman branch (d): r swapped to k, 1x1 at k    */
} orc_stats;

typedef struct orc_sym orc_sym;
typedef struct orc_num orc_num;

void orc_default_opts(orc_opts* o);

/* Symbolic analysis.  A is m x n CSC (sorted, no duplicates).  user_perm (length N, new->old)
 * may be NULL: then the oracle's own minimum-degree ordering is used.  The ordering is then
 * postordered (children visited in ascending order) and fundamental supernodes formed.   */
int orc_analyse(int m, int n, const int64_t* colptr, const int32_t* rowidx, int mode,
                const int32_t* user_perm, orc_sym** out);
/* Quadratic programs, AS mode only: the (1,1) block becomes -(Q + Theta^-1 + rho I).  Q is
 * n x n symmetric, given by its lower triangle in CSC (qcolptr n+1, rows >= the column and
 * strictly increasing; diagonal entries optional).  Q's couplings join the pattern. */
int orc_analyse_qp(int m, int n, const int64_t* colptr, const int32_t* rowidx,
                   const int64_t* qcolptr, const int32_t* qrowidx, const int32_t* user_perm,
                   orc_sym** out);
void orc_sym_free(orc_sym* S);
/* info: [N, nsuper, nnzL (incl. diagonal), maxfront, flops as int64] */
void orc_sym_info(const orc_sym* S, int64_t* info);
void orc_sym_perm(const orc_sym* S, int32_t* perm);       /* new -> old, length N        */
void orc_sym_parent(const orc_sym* S, int32_t* parent);   /* column etree, new numbering */
void orc_sym_colcount(const orc_sym* S, int64_t* cc);     /* |L column| incl. diagonal   */
void orc_sym_snptr(const orc_sym* S, int32_t* snptr);     /* nsuper+1                    */
void orc_sym_snparent(const orc_sym* S, int32_t* sp);     /* nsuper                      */
void orc_sym_front_rows(const orc_sym* S, int64_t* rowptr, int32_t* rows); /* nsuper+1, ... */

/* Numeric factorisation of K_static + E_dyn (Sections 3.2, 4.1, 4.5, 4.6). */
int orc_factorise(const orc_sym* S, const double* aval, const double* theta, double rho,
                  double delta, const orc_opts* o, orc_num** out);
/* The same for a quadratic program (qval: Q's lower values in the order of its pattern). */
int orc_factorise_qp(const orc_sym* S, const double* aval, const double* qval,
                     const double* theta, double rho, double delta, const orc_opts* o,
                     orc_num** out);
void orc_num_free(orc_num* F);
void orc_num_stats(const orc_num* F, orc_stats* st);
double orc_num_knorm(const orc_num* F);
/* Final pivot order: fperm[pos] = original variable; dense L (N x N col-major, positions),
 * D diagonal, D off-diagonal (at the first position of a 2x2), pivot type (0: 1x1,
 * 1: first of 2x2, 2: second), E_dyn at each position.  For small N only.               */
void orc_num_export(const orc_num* F, int32_t* fperm, double* Ldense, double* d, double* doff,
                    int8_t* ptype, double* edyn);
/* By position: the ORC_EF_* bits of the dynamic regularisation each 1x1 pivot received
 * (0 for 2x2 blocks). */
void orc_num_eflags(const orc_num* F, int8_t* eflag);

/* Solve with refinement (Sections 3, 4.5).  Column-major, leading dimension = rows.
 * NE: r7 (n x nrhs) may be NULL (zero); returns dx (n x nrhs) and dy (m x nrhs).
 * AS: returns dx, dy of the augmented system.  berr: per rhs, final normwise error;
 * steps: per rhs, refinement steps taken.                                              */
int orc_solve(const orc_sym* S, const orc_num* F, int nrhs, const double* r7,
              const double* r1, double* dx, double* dy, double* berr_nw, double* berr_cw,
              int* steps);

/* Residual and backward errors of x for the regularised system K_static x = b, computed
 * from A, Theta, rho, delta directly (Section 4.5).  b and x are N-vectors in the
 * system's own variables (AS: [x; y], N = n+m; NE: y, N = m).  r may be NULL.          */
int orc_residual(int m, int n, const int64_t* colptr, const int32_t* rowidx,
                 const double* aval, int mode, const double* theta, double rho,
                 double delta, const double* x, const double* b, double* r,
                 double* berr_nw, double* berr_cw, double* knorm);
/* The same with a quadratic program's Q (AS only; NULL pointers: an LP). */
int orc_residual_qp(int m, int n, const int64_t* colptr, const int32_t* rowidx,
                    const double* aval, int mode, const int64_t* qcolptr, const int32_t* qrowidx,
                    const double* qval, const double* theta, double rho, double delta,
                    const double* x, const double* b, double* r, double* berr_nw,
                    double* berr_cw, double* knorm);

/* Partial LDL^T of one dense front (Sections 4.4-4.6): f x f symmetric, column-major,
 * full storage, eliminating the first p pivots in windows of nb columns.  sigma: expected
 * pivot signs, shift: static regularisation per row (both permuted with the rows).
 * On exit F holds L in the first p columns (rows in pivoted order), the Schur complement
 * in F[p:, p:], perm[k] = original position now at position k (length f).            */
void orc_front_factor(int f, int p, double* F, int8_t* sigma, double* shift, int32_t* perm,
                      double knorm, const orc_opts* o, double* d, double* doff,
                      int8_t* ptype, double* edyn, orc_stats* st);

#ifdef __cplusplus
}
#endif
#endif
