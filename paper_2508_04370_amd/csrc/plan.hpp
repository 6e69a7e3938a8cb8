// Host-side symbolic plan: ordering, supernodal elimination tree, index maps and the
// level-by-level launch plan of the numeric factorisation and the solves.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace qdmf {

constexpr int NB = 64;  // pivot window width used by the device kernels
constexpr int SOLVE_BLOCK = 256;  // pivots per block of the multi-workgroup solves of big supernodes
// A trailing-update task (L_SYRK) packs into Task.k0 the first inner column k0 (a window start),
// the number of consecutive windows whose update it applies at once, less one, and whether it
// updates only the next window's columns (the narrow update inside a group of windows).  The
// tile origin is the end of the inner range: rows k1 + 64 a, columns k1 + 64 b.
constexpr int32_t SYRK_K0_MASK = (1 << 24) - 1;
constexpr int SYRK_COUNT_SHIFT = 24;  // three bits: up to SYRK_GROUP_MAX windows
constexpr int32_t SYRK_NARROW = 1 << 28;
constexpr int SYRK_GROUP_MAX = 4;

// One task of a batched launch.  Meaning per kernel:
//   small front / solve: s = supernode
//   window: s, k0 = window start, a = chunk of 64*npg rows below the window
//   finalize: s, k0 = first of 64 pivot columns
//   assemble: s, k0 = front column, [a, a+b) = range of its (child, child column) list
//   syrk:   s, k0 = packed inner range (below), a = row tile, b = column tile (64 rows each;
//           128 for L_SYRK128)
struct Task {
    int32_t s, k0, a, b;
};

enum LaunchKind : int32_t {
    L_SMALL = 0,     // whole front in LDS: assembly + factorisation
    L_ASSEMBLE = 1,  // large fronts: one workgroup per front column
    L_WINDOW = 2,    // pivot window: diagonal block + 64 panel rows per workgroup
    L_SYRK = 3,      // trailing update tiles
    L_FINALIZE = 4,  // factored diagonal blocks into place, row swaps of earlier columns
    L_SYRK128 = 7    // full trailing updates of large trailing matrices in 128 x 128 tiles
                     // (the number is its profiling kind; 5 and 6 are the solve passes)
};

struct Launch {
    int32_t kind;
    int32_t level;
    int64_t task0, ntask;  // range in the task array
    int32_t lds;           // dynamic LDS bytes (assembly)
    int32_t maxf;          // largest front order among the tasks
    int32_t npg = 0;       // window: panel row groups of 64 per workgroup (0 or 1)
    int64_t fin0 = 0, nfin = 0;  // trailing update: the level's finalize tasks run in the same launch
    int64_t nmix = 0;      // 128-tile trailing update: its first nmix tasks belong to fronts of
                           // order >= f_mix (FP32 products in mixed precision)
    int8_t stream = 0;     // 0: the library's stream; 1: the second (lookahead) stream, after
                           // the last pivot window enqueued before it on the first
    int8_t wait = 0;       // on the first stream: wait for the second stream's work so far
    double flops = 0;      // algorithmic work of the launch
    double bytes = 0;
};

// Solve launches of big supernodes (front order >= the split_solve_front option), spread over
// many workgroups (all right-hand sides at once).  Task fields per kind:
//   S_GATHER, S_FFIN, S_BLOAD, S_BSTORE: s, k0 = 256-row chunk of the front
//   S_FDIAG: s, k0 = pivot block j (SOLVE_BLOCK pivots);  S_BDIAG: s, k0 = j, [a, a + b) = its
//            partial sums
//   S_FUPD: s, k0 = j, a = 256-row chunk below the block
//   S_BPART: s, k0 = j, a = 256-row chunk below the block, b = index of its partial sums
enum SolveKind : int32_t { S_GATHER = 0, S_FDIAG, S_FUPD, S_FFIN, S_BLOAD, S_BPART, S_BDIAG, S_BSTORE };

struct SolveLaunch {
    int32_t kind;
    int64_t task0, ntask;
};

struct Plan {
    // problem
    int32_t m = 0, n = 0, mode = 0, N = 0;
    std::vector<int64_t> acp;   // A pattern, CSC
    std::vector<int32_t> ari;
    std::vector<int64_t> arp;   // A pattern, CSR: row pointers
    std::vector<int32_t> are;   // CSR -> CSC entry index
    std::vector<int32_t> acol;  // column of each CSC entry
    // quadratic programs (AS only): Q's lower triangle as given (CSC, n columns), and the full
    // symmetric pattern (CSC) with, per entry, the index of its value in the lower triangle;
    // per column the index of Q_jj or -1.  Empty for an LP.
    bool has_q = false;
    std::vector<int64_t> qcp;
    std::vector<int32_t> qri;
    std::vector<int64_t> qfcp, qfsrc, qdiag;
    std::vector<int32_t> qfri;

    // ordering (new -> old, old -> new) after postordering
    std::vector<int32_t> perm, iperm;

    // exact symbolic data (before amalgamation)
    int64_t nnz_l = 0;
    double flops_fact = 0, flops_solve = 0;

    // supernodes (after amalgamation), in postorder
    int32_t ns = 0;
    std::vector<int32_t> sn_ptr, sn_parent, sn_f, sn_p, sn_ld, sn_level, sn_nwin;
    std::vector<int64_t> sn_off;    // front offsets in the front arena (doubles)
    std::vector<int64_t> sn_rowptr; // row lists
    std::vector<int32_t> rows;      // global (new numbering) row index of each front row
    std::vector<int32_t> ch_ptr, ch;    // children, ascending
    std::vector<int64_t> rel_ptr;       // per supernode: CB rows mapped into parent front
    std::vector<int32_t> rel;
    std::vector<int64_t> ub_off;        // solve contribution buffer offset (per rhs column)
    std::vector<int64_t> fg_ptr;        // per front row (as rows[]): its forward-solve gather list
    std::vector<int64_t> fg_src;        // entries of the children's contribution buffers
    int64_t ub_total = 0;
    int64_t front_total = 0;            // doubles in the front arena
    int32_t max_front = 0, nlevels = 0;

    // entries of lower(K) grouped by new column: values are produced in this order
    std::vector<int64_t> kcol_ptr;      // N + 1
    std::vector<int32_t> kloc;          // row position inside the front of the column's supernode
    std::vector<int32_t> kcl;           // column position inside that front
    std::vector<int32_t> asm_child, asm_col;  // assembly lists of large-front columns
    std::vector<int32_t> krow_old, kcol_old;  // original indices of each entry (row >= col in new order)
    std::vector<int64_t> ksrc;          // AS: >= 0 A entry, -1-j primal diagonal j, -1-n-q entry q of Q's
                                        // lower triangle, KSRC_ZERO dual diagonal
    std::vector<int64_t> kpair_ptr;     // NE: per entry, pairs of A entries (a, b), column ascending
    std::vector<int32_t> kpair;         // 2 per pair
    // NE residual / norm: per original row, the K entries touching it
    std::vector<int64_t> krs_ptr;
    std::vector<int32_t> krs_ent, krs_other;

    std::vector<int8_t> primal_new;     // per new index: 1 if a primal (x) variable
    // AS: columns of A with more than LONG_COL entries (dense columns), summed by a workgroup
    // each in the residual and Krylov products; per column its index in long_col or -1
    std::vector<int32_t> long_col, long_of;

    // independent systems analysed together as one block-diagonal pattern (a batch); one
    // system otherwise.  K's original numbering: AS columns then rows, NE rows.
    int32_t nsys = 1;
    std::vector<int32_t> sys_col;       // per column of A
    std::vector<int32_t> sys_old;       // per K index, original numbering
    std::vector<int32_t> sys_new;       // per K index, elimination order
    std::vector<int64_t> sys_rng;       // per system: index ranges [a0, a1) and [b0, b1)
    std::vector<int64_t> sys_piv_ptr;   // per system: its pivot positions, ascending
    std::vector<int32_t> sys_piv;

    // launch plan
    std::vector<Task> tasks;
    std::vector<Launch> launches;       // factorisation, in order
    std::vector<int64_t> lvl_ptr;       // supernodes per level for the solves (nlevels + 1)
    std::vector<int32_t> lvl_sn;
    std::vector<double> lvl_solve_flops, lvl_solve_bytes;  // per level, one pass, one rhs
    std::vector<int32_t> lvl_small;     // per level: supernodes of lvl_sn solved one per workgroup (first)
    std::vector<int32_t> lvl_wave;      // per level: of those, the first ones, whose fronts have at
                                        // most 64 rows, are solved one per wavefront
    std::vector<Task> stasks;           // tasks of the big-supernode solve launches
    std::vector<int64_t> fwd_ptr, bwd_ptr;  // per level: its range of fwd_plan / bwd_plan
    std::vector<SolveLaunch> fwd_plan, bwd_plan;
    std::vector<int64_t> yoff;          // per supernode: rows in the solve work space (big only)
    // Inverses of the unit lower diagonal blocks (64 pivots each) of the supernodes that the
    // one-workgroup solve kernels handle: block j of supernode s is nb x nb, column-major, at
    // inv_off[s] + 4096 j (nb = 64 but for the last block); -1 where none.  One task
    // {s, j} per block.
    std::vector<int64_t> inv_off;
    int64_t inv_total = 0;
    std::vector<Task> inv_tasks;
    int64_t ytotal = 0;
    int64_t ppart_max = 0;              // most partial sums of one S_BPART launch

    int64_t device_bytes = 0;
};

constexpr int64_t KSRC_ZERO = INT64_MIN;
constexpr int64_t LONG_COL = 128;

struct AnalyseOptions {
    int ordering = 0;
    int grid[3] = {0, 0, 0};
    int amalgamate = 1;
    int small_front = 64;
    int split_solve_front = 1024;  // fronts at least this big: multi-workgroup solves
    int syrk_group_front = 1024;   // fronts at least this big: grouped trailing updates (0: none)
    int syrk_group = 4;            // windows per group
    int syrk_tile_front = 0;       // full trailing updates of at least this many rows: 128 x 128 tiles (0: never)
    int lookahead_front = 0;       // fronts at least this big: full updates past the next group's
                                   // columns on the second stream (0: none)
    int f_mix = 1024;              // mixed precision: fronts of at least this order take FP32 products
    const int32_t* user_perm = nullptr;
    // batch: nsys systems, system s owns columns [col_off[s], col_off[s+1]) and rows
    // [row_off[s], row_off[s+1]) of the block-diagonal A (nullptr: one system)
    int32_t nsys = 1;
    const int64_t* col_off = nullptr;
    const int64_t* row_off = nullptr;
    // quadratic programs (AS, one system): Q's lower triangle, CSC with n columns
    const int64_t* q_colptr = nullptr;
    const int32_t* q_rowidx = nullptr;
};

// Approximate minimum degree ordering of a symmetric pattern given as full adjacency
// (CSR, no diagonal).  Returns order[k] = node eliminated k-th.
void amd_order(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
               std::vector<int32_t>& order);

// Factorisation flops sum_j c_j (c_j + 3) of an ordering of a symmetric pattern, and the
// same plus a charge for the height of its elimination tree (sequential pivot steps).
double order_flops(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
                   const std::vector<int32_t>& order);
double order_cost(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
                  const std::vector<int32_t>& order);

// Multilevel graph nested dissection of the same kind of pattern; order[k] = node k-th.
void nd_order(int32_t N, const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
              std::vector<int32_t>& order);

// Geometric nested dissection for grid-coupled problems (rows on an nx x ny x nz grid).
void grid_nd_order(const Plan& P, const int grid[3], const std::vector<int64_t>& xadj,
                   const std::vector<int32_t>& adj, std::vector<int32_t>& order);

// Builds the whole plan.  Returns 0 or a QDMF_ERR_* code; msg explains failures.
// Lower entries (with the diagonal) of the pattern of A A^T, counted row by row; stops and
// returns a value above `limit` as soon as the count exceeds it.
int64_t ne_pattern_count(int32_t m, int32_t n, const int64_t* colptr, const int32_t* rowidx, int64_t limit);

int build_plan(int32_t m, int32_t n, const int64_t* colptr, const int32_t* rowidx,
               int32_t mode, const AnalyseOptions& opt, Plan& P, std::string& msg);

}  // namespace qdmf
