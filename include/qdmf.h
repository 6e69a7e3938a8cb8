/*
 * qdmf -- multifrontal LDL^T factorise + solve of the regularised Newton systems of an LP
 * interior point method, on one AMD Instinct MI355X (gfx950).
 *
 * The problem statement follows Zanetti & Gondzio, arXiv 2508.04370:
 *   normal equations (NE), Section 3 eq. (normeq) with (regul_matrix):
 *       K = A (Theta^{-1} + rho I)^{-1} A^T + delta I            (order m)
 *   augmented system (AS), Section 3 eq. (augsys) with (regul_matrix):
 *       K = [[-(Theta^{-1} + rho I), A^T], [A, delta I]]         (order n + m)
 * A is m x n and fixed across IPM iterations; Theta (diagonal, n, positive) changes every
 * iteration.  Ordering and symbolic analysis run once (Section 4.2); the numeric
 * factorisation (Section 4.1, pivoting and regularisation of Sections 4.5-4.6) and the
 * solves with iterative refinement (Section 4.5) run on the GPU each iteration.
 *
 * Conventions
 *   - return value 0: success; < 0: error (nothing was enqueued); > 0: numerical warning.
 *   - indices are int32, offsets int64.  Column-major dense vectors, leading dim = rows.
 *   - pointers documented "device" must be device memory of the handle's device.
 *   - a handle is not thread-safe; separate handles are independent.
 *   - factorise / graph_launch are asynchronous on the handle's stream; solve is
 *     asynchronous up to its refinement decisions (see qdmf_solve); analyse, symbolic,
 *     the stats calls and destroy synchronise.
 */
#ifndef QDMF_H
#define QDMF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qdmf_ctx* qdmf_handle;

enum { QDMF_NE = 0, QDMF_AS = 1 };              /* system form (Section 3)           */
enum { QDMF_FP64 = 0, QDMF_MIXED = 1 };         /* precision of the Schur updates    */
#define QDMF_NOALLOC_SCRATCH_BYTES 67108864      /* qdmf_solve_noalloc work space per GPU (64 MiB) */
enum { QDMF_ORDER_AMD = 0, QDMF_ORDER_USER = 1, QDMF_ORDER_GRID_ND = 2, QDMF_ORDER_ND = 3, QDMF_ORDER_AUTO = 4 };
/* kernel kinds for qdmf_profile_kind */
enum {
    QDMF_K_SMALL = 0,    /* small fronts: assembly + factorisation in LDS        */
    QDMF_K_ASSEMBLE = 1, /* large fronts: extend-add, one workgroup per column   */
    QDMF_K_WINDOW = 2,   /* pivot window: diagonal block + panel rows            */
    QDMF_K_SYRK = 3,     /* trailing Schur update on MFMA                        */
    QDMF_K_FINALIZE = 4, /* factored blocks into place, row swaps                */
    QDMF_K_FWD = 5,      /* forward substitution + D, one tree level             */
    QDMF_K_BWD = 6,      /* backward substitution, one tree level                */
    QDMF_K_SYRK128 = 7   /* trailing Schur update of large trailing matrices,
                            128 x 128 tiles on MFMA                               */
};

enum {
    QDMF_OK = 0,
    QDMF_ERR_INVALID_ARG = -1,    /* bad argument, bad CSC, Theta <= 0 or not finite     */
    QDMF_ERR_HIP = -2,            /* a HIP runtime call failed                            */
    QDMF_ERR_OOM = -3,            /* memory plan exceeds the cap or hipMalloc failed     */
    QDMF_ERR_INDEX_OVERFLOW = -4, /* a 32-bit index would overflow (Section 5.4 lesson)   */
    QDMF_ERR_NOT_ANALYSED = -5,
    QDMF_ERR_NOT_FACTORISED = -6,
    QDMF_ERR_NO_MATRIX = -7,      /* qdmf_set_matrix not called                          */
    QDMF_ERR_UNSUPPORTED = -8,    /* e.g. a front larger than the kernels support        */
    QDMF_WARN_DYN_REG = 1,        /* dynamic regularisation (Prop. 3 / sign rule) fired   */
    QDMF_WARN_INERTIA = 2,        /* inertia differs from the quasi-definite one          */
    QDMF_WARN_NOT_CONVERGED = 3,  /* refinement stopped above the target backward error  */
    QDMF_WARN_LARGE_REG = 4       /* some |E_dyn| > tau_big * ||K||_1 (Section 4.6)       */
};

typedef struct {
    int32_t nb;               /* pivot window width; numerical parameter (Section 4.4), 64  */
    double alpha;             /* Bunch-Kaufman constant (Section 4.5), (1+sqrt(17))/8       */
    double eps_lift;          /* lift threshold factor (Section 4.5), 2^-52                 */
    int32_t presort;          /* swap the largest diagonal first (Section 4.5), 1           */
    int32_t max_refine;       /* refinement steps, FP64 path (Section 4.5), 2               */
    int32_t max_refine_mixed; /* refinement steps, mixed path, 3 (each a GMRES correction of
                                 up to 3 Krylov steps preconditioned by the factor)        */
    double target_berr;       /* normwise backward error target, FP64 path, 1e-12          */
    double target_berr_mixed; /* normwise backward error target, mixed path, 1e-10         */
    double tau_big;           /* "too large" regularisation threshold (Section 4.6), 1e-8  */
    int32_t ordering;         /* QDMF_ORDER_* (default AUTO: the cheaper of AMD and ND)     */
    int32_t grid[3];          /* GRID_ND: row grid dims, row r = x + g0*(y + g1*z)          */
    int32_t amalgamate;       /* relaxed supernode amalgamation (Section 4.1), 1            */
    int32_t f_mix;            /* MIXED: fronts of order >= f_mix use FP32 Schur updates    */
    int32_t small_front;      /* fronts of order <= small_front are factorised in LDS, 64  */
    int64_t mem_cap_bytes;    /* 0: none; analyse fails with QDMF_ERR_OOM above it         */
    int32_t split_solve_front; /* fronts of order >= this are solved by many workgroups per
                                  step, all right-hand sides together, and so are the fronts
                                  of at least min(128, this) rows on the same tree level with
                                  no more 64-pivot blocks; the rest by one workgroup each;
                                  >= 1, 1024                                               */
    int32_t syrk_group_front; /* fronts of order >= this (0: none) apply the Schur update of
                                 syrk_group consecutive pivot windows to their trailing
                                 matrix at once (the columns of each next window of the
                                 group are updated as soon as it is reached); 1024        */
    int32_t syrk_group;       /* windows per such group, 1..4; 4                           */
    int32_t syrk_tile_front;  /* full trailing updates (after a window, or after a group's last
                                 window) of trailing matrices of at least this many rows run
                                 in 128 x 128 tiles instead of 64 x 64 (0: never); 0        */
    int32_t mixed_check;      /* MIXED: which systems are factorised again in FP64: 0 none,
                                 1 those with a pivot that is not finite, 2 also those with
                                 some |E_dyn| > tau_big ||K||_1, 3 also those with any
                                 Proposition 3 or sign-rule pivot; 2                         */
    int32_t lookahead_front;  /* fronts of order >= this (0: none) overlap their trailing
                                 updates with the next pivot windows (Section 4.4's blocked
                                 factorisation): the tiles of a full update beyond the next
                                 group's pivot columns run on a second stream the library
                                 owns, joined back into the caller's stream before any work
                                 that reads them and before the factorisation ends; the
                                 factor is bitwise the same as with 0.  Measured no faster
                                 here: the update tiles and the window kernel cannot share
                                 a compute unit's registers, so each slows the other; 0     */
    int32_t graph_poll;       /* 1: a captured graph is cut at the refinement decisions, and
                                 qdmf_graph_launch reads their flags on the host between the
                                 parts, as eager solves do, launching only the refinement and
                                 Krylov steps some right-hand side still needs; 0: one graph
                                 holding every step (finished steps return at once), launched
                                 without any host read; 1                                  */
} qdmf_options;

typedef struct {
    int32_t N;                /* order of K                                                 */
    int32_t nsuper;           /* number of supernodes                                       */
    int32_t nlevels;          /* levels of the supernodal tree (leaves = 0)                 */
    int32_t max_front;        /* largest front order                                        */
    int64_t nnz_l;            /* nonzeros of L (exact structure, incl. diagonal)            */
    int64_t nnz_k;            /* nonzeros of lower(K)                                       */
    double flops_fact;        /* sum_j c_j (c_j + 3), exact structure                       */
    double flops_solve;       /* 4 sum_j c_j + N per right-hand side                        */
    int64_t device_bytes;     /* bytes the handle holds on the device                       */
    int64_t front_bytes;      /* of which dense front storage                               */
    /* arrays owned by the handle, valid until the next analyse or destroy (host memory) */
    const int32_t* perm;      /* new -> old, length N                                       */
    const int32_t* sn_ptr;    /* supernode s = columns [sn_ptr[s], sn_ptr[s+1]), nsuper+1   */
    const int32_t* sn_parent; /* parent supernode or -1, nsuper                             */
    const int32_t* sn_front;  /* front order f of each supernode, nsuper                    */
    const int32_t* sn_level;  /* level of each supernode, nsuper                            */
} qdmf_symbolic_info;

typedef struct {
    int64_t nneg, npos, nzero;        /* inertia of D                                       */
    int64_t n2x2, nlift, nprop3, nsign, nzskip;
    double max_edyn;                  /* max |E_dyn|                                        */
    double knorm;                     /* ||K_static||_1                                     */
    int32_t status;                   /* 0 or the first QDMF_WARN_* that applies            */
    int32_t nredo_fp64;               /* mixed precision: systems factorised again in FP64  */
} qdmf_factor_info;

typedef struct {
    int32_t nrhs;
    int32_t max_steps;                /* max over right-hand sides of refinement steps      */
    double berr_nw;                   /* max over right-hand sides, final normwise error   */
    double berr_cw;                   /* max over right-hand sides, componentwise error    */
    double berr_nw_initial;           /* before refinement                                  */
    int32_t status;                   /* 0 or QDMF_WARN_NOT_CONVERGED                       */
} qdmf_solve_info;

/* Fills *opt with the defaults listed above. */
void qdmf_default_options(qdmf_options* opt);

/* Creates a handle bound to `device` and the HIP stream `hip_stream` (NULL: the null
 * stream).  opt may be NULL (defaults); it is copied.  Owns every device allocation it
 * makes.  Errors: QDMF_ERR_INVALID_ARG, QDMF_ERR_HIP. */
int qdmf_create(qdmf_handle* h, int device, void* hip_stream, const qdmf_options* opt);

/* Rebinds the stream used by later asynchronous calls. */
int qdmf_set_stream(qdmf_handle h, void* hip_stream);

/* Symbolic analysis of the pattern of A (Section 4.2: ordering and symbolic factorisation
 * once, reused every iteration; Section 4.3: supernodal elimination tree).  Host arrays
 * (m, n >= 0; colptr: n+1 entries; rowidx: sorted strictly increasing within each column)
 * are read and not retained.  user_perm (new -> old, length N) is used when
 * opt.ordering == QDMF_ORDER_USER and ignored otherwise (may be NULL).  Runs on the host,
 * then uploads the plan.  Errors: QDMF_ERR_INVALID_ARG (bad CSC / perm),
 * QDMF_ERR_OOM (plan above mem_cap_bytes or allocation failure), QDMF_ERR_INDEX_OVERFLOW,
 * QDMF_ERR_UNSUPPORTED. */
int qdmf_analyse(qdmf_handle h, int32_t m, int32_t n, const int64_t* colptr,
                 const int32_t* rowidx, int32_t mode, const int32_t* user_perm);

/* Quadratic programs (the extension of the augmented system to min c^T x + x^T Q x / 2 that
 * the paper names beside its LP method): the (1,1) block of the augmented system becomes
 * -(Q + Theta^-1 + rho I), so K_static = [[-(Q + Theta^-1 + rho I), A^T], [A, delta I]].
 * For positive semidefinite Q the matrix stays quasidefinite (Section 4.6), and the pivoting,
 * the regularisation and the expected inertia (n negative, m positive) are those of the LP.
 * Analyses the pattern of A together with Q's couplings (x_j -- x_k where Q_jk != 0), in
 * QDMF_AS mode for one system.  Q (n x n, symmetric) is given by its lower triangle in CSC
 * (q_colptr: n+1 entries; q_rowidx: rows >= the column, strictly increasing; diagonal
 * entries optional); host arrays, read and not retained.  Other arguments as qdmf_analyse.
 * Errors: as qdmf_analyse, and QDMF_ERR_INVALID_ARG for a bad Q pattern. */
int qdmf_analyse_qp(qdmf_handle h, int32_t m, int32_t n, const int64_t* colptr,
                    const int32_t* rowidx, const int64_t* q_colptr, const int32_t* q_rowidx,
                    const int32_t* user_perm);

/* Values of Q's lower triangle in the order of the pattern given to qdmf_analyse_qp (FP64;
 * host memory if on_device == 0, else device memory).  Copied; must be called before the
 * first factorisation of a quadratic program.  Errors: QDMF_ERR_NOT_ANALYSED,
 * QDMF_ERR_INVALID_ARG (also when the analysed problem has no Q). */
int qdmf_set_hessian(qdmf_handle h, const double* q_val, int32_t on_device);

/* Symbolic results (host memory owned by the handle).  Error: QDMF_ERR_NOT_ANALYSED. */
int qdmf_symbolic(qdmf_handle h, qdmf_symbolic_info* out);

/* Values of A in the order of the analysed pattern (nnz entries, FP64); host memory if
 * on_device == 0, else device memory.  Copied; call again whenever A's values change.
 * Errors: QDMF_ERR_NOT_ANALYSED, QDMF_ERR_INVALID_ARG. */
int qdmf_set_matrix(qdmf_handle h, const double* a_val, int32_t on_device);

/* Numeric factorisation P (K_static + E_dyn) P^T = L D L^T on the device (Sections 4.1,
 * 4.4-4.6).  theta_dev: device, n entries, positive and finite (checked on the device:
 * a bad value makes qdmf_factor_stats return QDMF_ERR_INVALID_ARG); it must stay valid
 * until the stream reaches this call's end.  rho, delta >= 0 are the static
 * regularisations.  prec: QDMF_FP64 or QDMF_MIXED (FP32 MFMA Schur updates on fronts of
 * order >= opt.f_mix; everything else FP64).  In mixed precision a system whose factor
 * then shows a breakdown of the FP32 updates (opt.mixed_check: by default a pivot that is
 * not finite or a dynamic regularisation above tau_big ||K||_1) is factorised again in FP64,
 * and only that system; qdmf_factor_info.nredo_fp64 counts them.  Executed eagerly, this
 * call then waits for the stream to read that count.  When no front of order >= f_mix has a
 * trailing update, a mixed factorisation is the FP64 one: no check, and its solves refine by
 * plain FP64 corrections (to the mixed target).  L, D are owned by the handle.
 * Returns < 0 only for argument errors; numerical outcomes come from qdmf_factor_stats.
 * An empty system (m + n == 0) launches nothing and reports zero pivots. */
int qdmf_factorise(qdmf_handle h, const double* theta_dev, double rho, double delta,
                   int32_t prec);

/* Solves K_static [dx; dy] = [r7; r1] (AS) or K_static dy = r1 + A theta~ r7 and
 * dx = theta~ (A^T dy - r7) (NE, Section 3 eq. (normeq)), then refines in FP64 against
 * K_static until the normwise backward error reaches the target or the step limit
 * (Section 4.5).  All vectors are device memory, column-major: r7 and dx n x nrhs, r1 and
 * dy m x nrhs; r7 may be NULL (zero).  Outputs must not alias inputs.  A correction of
 * the FP64 path is d = (L D L^T)^{-1} r; of the mixed path, GMRES on K_static (L D L^T)^{-1}
 * with at most 8 Krylov steps, its small dense part and stop flags on the device.  Between
 * refinement steps (and between Krylov steps) the call waits for the stream to read the
 * device's stop flags and launches no further step once every right-hand side is done;
 * under graph capture (qdmf_graph_capture) it waits for nothing and enqueues every step,
 * whose kernels then return at once for finished right-hand sides: both compute the same
 * result.  An empty system (m + n == 0) launches nothing and reports zero backward error.
 * Errors: QDMF_ERR_NOT_FACTORISED, QDMF_ERR_INVALID_ARG. */
int qdmf_solve(qdmf_handle h, int32_t nrhs, const double* r7_dev, const double* r1_dev,
               double* dx_dev, double* dy_dev);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): qdmf_solve with the same arguments, result and
 * statistics, whose work space (QDMF_NOALLOC_SCRATCH_BYTES of device memory per GPU, a
 * fixed array that each GPU the library runs on holds until the process ends) is not
 * allocated: it calls no hipMalloc, hipFree or allocating library routine and never reads
 * the device's flags from the host (it enqueues every refinement step, as under graph
 * capture).  The factorisation must exist (qdmf_factorise: the handle's own memory).  Every
 * call on one GPU shares that GPU's array and leaves the last call's contents in it, so calls
 * that overlap on one GPU (other streams, other threads, other handles) race; calls ordered
 * on one stream do not.  Errors: as qdmf_solve; QDMF_ERR_OOM (nothing launched) when the
 * work space of nrhs right-hand sides (the solve vectors and, after a mixed factorisation,
 * the Krylov basis) exceeds QDMF_NOALLOC_SCRATCH_BYTES; QDMF_ERR_HIP when the array's
 * address could not be found on this device. */
int qdmf_solve_noalloc(qdmf_handle h, int32_t nrhs, const double* r7_dev, const double* r1_dev,
                       double* dx_dev, double* dy_dev);

/* ---- batches of independent systems ---------------------------------------------------
 * A batch of count independent LPs of one mode is analysed as one block-diagonal pattern:
 * system q's column j becomes column col_off[q] + j and its row i row row_off[q] + i (offsets
 * from qdmf_batch_offsets), so every tree-level launch of the factorisation and the solves
 * covers the fronts of all systems at once (the many-small-fronts case of Section 4.3's tree
 * parallelism).  Each system keeps its own ||K_static||_1 (lift threshold, Section 4.5), its
 * own rho and delta, its own backward errors and refinement decisions, and its own inertia.
 * After qdmf_batch_analyse: qdmf_set_matrix takes the systems' values concatenated in system
 * order; qdmf_factorise (one rho, delta for all) or qdmf_batch_factorise (per system);
 * qdmf_solve on concatenated vectors (r7, dx: sum n; r1, dy: sum m); qdmf_solve_stats reports
 * the worst system per right-hand side and qdmf_batch_stats every system. */

/* m, n, colptr, rowidx: count entries each (host), one CSC pattern per system as for
 * qdmf_analyse.  Orderings QDMF_ORDER_USER and QDMF_ORDER_GRID_ND are not accepted.
 * Errors: as qdmf_analyse. */
int qdmf_batch_analyse(qdmf_handle h, int32_t count, const int32_t* m, const int32_t* n,
                       const int64_t* const* colptr, const int32_t* const* rowidx, int32_t mode);

/* row_off, col_off: count + 1 entries each (host; either may be NULL).  For a single system
 * they are {0, m} and {0, n}.  Errors: QDMF_ERR_NOT_ANALYSED. */
int qdmf_batch_offsets(qdmf_handle h, int64_t* row_off, int64_t* col_off);

/* As qdmf_factorise with rho[q], delta[q] (host, count entries, >= 0) for system q.  The
 * call waits for the stream before it stages the shifts (graph capture is not supported for
 * this call: qdmf_batch_factorise_dev and qdmf_batch_graph_capture take the shifts from device
 * memory). */
int qdmf_batch_factorise(qdmf_handle h, const double* theta_dev, const double* rho,
                         const double* delta, int32_t prec);

/* As qdmf_batch_factorise with rho_dev[q], delta_dev[q] (device, count doubles each, read when
 * the factorisation runs; the caller keeps them until then): nothing is staged on the host
 * and the call does not wait for the stream, so a graph may capture it.  A negative or
 * non-finite shift is found on the device and reported as invalid input by
 * qdmf_factor_stats, as an invalid Theta is.  Errors: as qdmf_batch_factorise. */
int qdmf_batch_factorise_dev(qdmf_handle h, const double* theta_dev, const double* rho_dev,
                             const double* delta_dev, int32_t prec);

/* Synchronises; any pointer may be NULL.  inertia: 3 x count (negative, positive, zero
 * pivots of system q at 3q..3q+2); berr_nw, steps: count x nrhs of the last solve, entry
 * r * count + q for right-hand side r of system q.  Errors: QDMF_ERR_NOT_FACTORISED. */
int qdmf_batch_stats(qdmf_handle h, int64_t* inertia, double* berr_nw, int32_t* steps);

/* Synchronises the stream and reports the last factorisation.  Returns the status (0,
 * a QDMF_WARN_* code, or QDMF_ERR_INVALID_ARG if Theta was invalid). */
int qdmf_factor_stats(qdmf_handle h, qdmf_factor_info* out);

/* Synchronises the stream and reports the last solve.  berr_nw_per_rhs and
 * steps_per_rhs may be NULL, else nrhs entries (host).  Returns 0 or
 * QDMF_WARN_NOT_CONVERGED. */
int qdmf_solve_stats(qdmf_handle h, qdmf_solve_info* out, double* berr_nw_per_rhs,
                     int32_t* steps_per_rhs);

/* Dense-factor export for tests and inspection (host memory, synchronises).
 * pivot_order: length N, original variable at each final pivot position;
 * d, doff: D diagonal and 2x2 off-diagonals by position; ptype: 0 1x1, 1/2 first/second
 * of a 2x2 block; edyn: dynamic regularisation added at each position (Section 3.2);
 * any pointer may be NULL. */
int qdmf_export_d(qdmf_handle h, int32_t* pivot_order, double* d, double* doff,
                  int8_t* ptype, double* edyn);

/* Dynamic regularisation of each pivot position (host memory, N bytes, synchronises): bit 0
 * a lift (Section 4.5: both the pivot and its column below tiny), bit 1 Proposition 3
 * (Section 4.6: the pivot raised to beta), bit 2 the sign rule (Section 4.6: the pivot
 * forced to its expected sign); 0 for positions of 2x2 blocks and unmodified pivots.
 * Positions as in qdmf_export_d.  Errors: QDMF_ERR_NOT_FACTORISED, QDMF_ERR_INVALID_ARG. */
int qdmf_export_flags(qdmf_handle h, uint8_t* flags);

/* Copies supernode s's factored front columns (f x p panel of L, rows in the front's
 * pivoted order, ld = f) and its row list (global original indices, length f) to host. */
int qdmf_export_front(qdmf_handle h, int32_t s, double* panel, int32_t* rows);

/* Captures factorise + nsolves x solve (each with refinement) once as a HIP graph; later
 * qdmf_graph_launch replays it on the handle's stream, reading Theta and the right-hand
 * sides from the same device buffers (the caller refreshes them in place).  Capturing runs
 * nothing and leaves the handle's factorisation and solve state as they were; a launch makes
 * it the graph's (the stats and export calls then report the replayed factorisation and
 * solves).  The result of a replay equals that of the same calls made eagerly.
 * With the option graph_poll (default) the capture is cut into parts at the points where an
 * eager solve reads its refinement flags (each refinement pass, each Krylov step after the
 * first, the FP64 redo of a mixed factorisation that broke down); qdmf_graph_launch then
 * launches the parts in order and, before a conditional part, copies its flags to pinned
 * host memory and waits for the stream, skipping the part (and the rest of its loop) when
 * no unit needs it.  With graph_poll = 0 the capture is one graph that holds every step and
 * qdmf_graph_launch only enqueues it.
 * Errors: QDMF_ERR_HIP, QDMF_ERR_NOT_ANALYSED, QDMF_ERR_INVALID_ARG (also for an empty
 * system, which has nothing to capture), QDMF_ERR_OOM (the pinned flag buffer). */
int qdmf_graph_capture(qdmf_handle h, const double* theta_dev, double rho, double delta,
                       int32_t prec, int32_t nsolves, int32_t nrhs, const double* r7_dev,
                       const double* r1_dev, double* dx_dev, double* dy_dev);
int qdmf_graph_launch(qdmf_handle h);

/* qdmf_graph_capture for a batch with per-system shifts: rho_dev[q], delta_dev[q] (device,
 * count doubles each) are read by every replay, so the caller refreshes them in place as it
 * does Theta (Section 4.6's regularisation may then change per system and iteration).
 * Errors: as qdmf_graph_capture. */
int qdmf_batch_graph_capture(qdmf_handle h, const double* theta_dev, const double* rho_dev,
                             const double* delta_dev, int32_t prec, int32_t nsolves,
                             int32_t nrhs, const double* r7_dev, const double* r1_dev,
                             double* dx_dev, double* dy_dev);

/* Measurement hook: while kind >= 0, every later eager launch of that kernel kind (above)
 * is bracketed by a pair of HIP events recorded on the handle's stream; kind = -1 stops.
 * Not applied inside qdmf_graph_capture.  Errors: QDMF_ERR_INVALID_ARG. */
int qdmf_profile_kind(qdmf_handle h, int32_t kind);

/* Synchronises the stream and returns, for the launches timed since the last read: their
 * number, the sum of their durations (ms, from the events), and their algorithmic flops and
 * bytes (from the symbolic structure: the work each launch must do, independent of how).
 * Resets the counters.  Any pointer may be NULL. */
int qdmf_profile_read(qdmf_handle h, int64_t* launches, double* total_ms, double* flops,
                      double* bytes);

/* Measurement: the peaks the roofline fractions are also reported against, measured on
 * `device` with events on `hip_stream`: FP64 and FP32 16x16x4 matrix instructions (the trailing
 * update's) in TFLOP/s, independent FP64 vector FMAs in TFLOP/s, and a streaming device copy of
 * 1 GiB (2 GiB moved) in GB/s; best of a few runs each.  Allocates and frees 2 GiB + 2 MiB of
 * device memory and synchronises the stream.  Any pointer may be NULL.
 * Errors: QDMF_ERR_HIP, QDMF_ERR_OOM. */
int qdmf_peak_probe(int device, void* hip_stream, double* mfma_f64_tflops, double* mfma_f32_tflops,
                    double* valu_f64_tflops, double* hbm_gbs);

/* Choice between the normal equations and the augmented system for the pattern of A
 * (Section 4.2: both can be analysed and the better taken, the augmented system first, and
 * the normal equations given up as soon as forming their pattern would hold more entries than
 * the augmented system's factor; Section 1: dense columns rule the normal equations out).
 * A column is dense when it holds at least max(64, ceil(m / 10)) entries.  When the normal
 * equations survive, both are analysed with the handle's options and the one with fewer
 * predicted factorisation flops is chosen (ties: NE).  Host only; the handle's own analysis
 * is not changed.  Inputs as for qdmf_analyse.  Errors: QDMF_ERR_INVALID_ARG,
 * QDMF_ERR_INDEX_OVERFLOW, QDMF_ERR_UNSUPPORTED. */
typedef struct {
    int32_t mode;             /* QDMF_NE or QDMF_AS                                          */
    int32_t ndense;           /* dense columns of A                                          */
    int32_t ne_abandoned;     /* 1: the normal equations were given up before their analysis  */
    int64_t nnz_l_as;         /* nnz(L) of the augmented system                              */
    int64_t nnz_ne_pattern;   /* lower entries (with the diagonal) of the pattern of A A^T,
                                 counted up to the point where it was given up               */
    int64_t nnz_l_ne;         /* nnz(L) of the normal equations, -1 if not analysed           */
    double flops_as, flops_ne; /* predicted factorisation flops; flops_ne -1 if not analysed */
} qdmf_mode_choice;
int qdmf_choose_mode(qdmf_handle h, int32_t m, int32_t n, const int64_t* colptr,
                     const int32_t* rowidx, qdmf_mode_choice* out);

/* Interior point driver around the factorise and solve calls (Section 3: Newton system
 * reduced to the augmented system, predictor with sigma = 0, centrality correctors from the
 * complementarity products at the trial point, steps to the boundary, the termination test of
 * Section 3.1; Section 4.7: the number of correctors).  LP of Section 2:
 *     min c^T x  subject to  A x = b,  l <= x <= u,
 * with slacks x^l = x - l, x^u = u - x and multipliers z^l, z^u.  Every l_j must be finite
 * (no free variables, as the paper assumes); u_j is finite and above l_j, or +inf.  A is the
 * matrix of the handle, which must be analysed in QDMF_AS mode with qdmf_set_matrix called.
 * Start: x = l + 1 (the midpoint of [l, u] where u - l < 2), z^l = 1, z^u = 1 where u is
 * finite, y = 0.
 * Arguments (caller-owned device buffers): b (m), c (n); l (n) or NULL for l = 0; u (n) or
 * NULL for u = +inf everywhere; x, z^l (n) and y (m) receive the last iterate; zu (n) receives
 * z^u (0 where u is infinite) or is NULL.  Runs on the handle's stream and synchronises it
 * several times per iteration.  A handle analysed with qdmf_analyse_qp (Q set with
 * qdmf_set_hessian) solves the quadratic program min c^T x + x^T Q x / 2 under the same
 * constraints: the dual residual gains +Q x, the factorised block is -(Q + Theta^-1 + rho I)
 * and both objectives carry x^T Q x / 2.  Errors: QDMF_ERR_INVALID_ARG (also for a bad bound
 * and for m == 0 or n == 0),
 * QDMF_ERR_NOT_ANALYSED (or not AS), QDMF_ERR_NO_MATRIX, QDMF_ERR_HIP, QDMF_ERR_OOM, and the
 * codes of qdmf_factorise / qdmf_solve. */
typedef struct {
    double tau;               /* feasibility and optimality tolerance (Section 3.1), 1e-8     */
    double rho, delta;        /* static regularisation of every factorisation (Section 3.2),
                                 1e-10 and 1e-10                                              */
    int32_t max_iter;         /* 100                                                         */
    int32_t correctors;       /* 0: Section 4.7's estimate; > 0: this many per iteration     */
    int32_t kmax;             /* most correctors from the estimate, 6                        */
    double alpha_f;           /* factorisation-efficiency factor of that estimate, 0.025     */
    int32_t prec;             /* QDMF_FP64 or QDMF_MIXED for every factorisation             */
} qdmf_ipm_options;

typedef struct {
    int32_t status;           /* 0: optimal; QDMF_WARN_NOT_CONVERGED: iteration limit         */
    int32_t iters;            /* iterations taken (factorisations)                           */
    int32_t correctors;       /* correctors allowed per iteration                            */
    double primal_obj, dual_obj;
    double pinf;              /* max of ||b - A x||_inf, ||l - x + x^l||_inf, ||u - x - x^u||_inf */
    double dinf;              /* ||c - A^T y - z^l + z^u (+ Q x)||_inf                       */
    double mu;                /* mean complementarity product at the last iterate            */
    double ms;                /* wall time of the iterations                                 */
} qdmf_ipm_info;

void qdmf_ipm_default_options(qdmf_ipm_options* opt);

/* history: NULL or room for 4 * max_iter doubles; per iteration it receives mu, alpha_p,
 * alpha_d and the number of correctors used. */
int qdmf_ipm_solve(qdmf_handle h, const double* b_dev, const double* c_dev, const double* l_dev,
                   const double* u_dev, double* x_dev, double* y_dev, double* zl_dev, double* zu_dev,
                   const qdmf_ipm_options* opt, qdmf_ipm_info* info, double* history);

/* Frees everything the handle owns.  NULL is ignored. */
void qdmf_destroy(qdmf_handle h);

/* Static string for a status code. */
const char* qdmf_status_string(int code);

/* Human-readable detail of the last failure of a handle's analyse or allocation (owned by
 * the handle; empty if none). */
const char* qdmf_last_message(qdmf_handle h);

#ifdef __cplusplus
}
#endif
#endif
